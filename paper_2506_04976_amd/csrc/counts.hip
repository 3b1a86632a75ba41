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

// Geometry of one bin with counts within its line (plane p, TOF bin b): the
// sample rows [is, ie] (z range, then TOF window), the table position
// pos(i) = pA i + pB of row i, the padded axial position u(i) = zA i + zB
// and the step length ell.
struct RecGeo {
    int is, ie;
    float pA, pB, zA, zB, ell;
};

template <bool TOF>
__device__ __forceinline__ RecGeo rec_geo(const ProjArgs &a, const CountArgs &c, const LineP &L, const PlaneP &P,
                                          int b) {
    RecGeo r;
    const float len = sqrtf(L.lt2 + P.dz2);
    r.ell = L.vm_um * len;
    z_clip<true>(L, P, a.nz, r.is, r.ie);  // (u is clamped by the loops)
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
    // Rows whose axial position u would leave the sheet row (cells j, j + 1
    // for u in [0, rz - 1)) or whose table position would leave the TOF table
    // carry no weight (zero padding, outside the TOF support): drop them at the
    // ends, so that the line kernels need no clamps.  Both positions are affine
    // in the row and evaluated as the kernels do (one correctly rounded FMA,
    // monotone in the row), so rows between two in-range ends are in range.
    const float ulim = (float)(a.rz - 1);
    auto in_range = [&](int i) {
        const float u = fmaf((float)i, r.zA, r.zB);
        if (!(u >= 0.f && u < ulim)) return false;
        if (TOF) {
            const float pos = fmaf((float)i, r.pA, r.pB);
            if (!(pos >= 0.f && pos <= c.pos_max)) return false;
        }
        return true;
    };
    while (r.is <= r.ie && !in_range(r.is)) ++r.is;
    while (r.is <= r.ie && !in_range(r.ie)) --r.ie;
    return r;
}

// Compaction of one line's bins with y > 0, TOF bin major (then plane): the
// records that share a wave then have TOF windows at the same place along the
// line, so their sample loops run for about the same number of rows.  Each
// record carries its LOR's geometry (rec_geo), so that the line kernels load
// one record per bin and nothing else.
template <bool TOF>
__global__ void __launch_bounds__(256) k_counts_fill(const void *__restrict__ y, int dt, const float *__restrict__ add,
                                                     const float *__restrict__ mult, int64_t bins_per_line,
                                                     const int64_t *__restrict__ line_off, ProjArgs a, CountArgs c,
                                                     CountRec *__restrict__ items) {
    __shared__ int s_w[4];
    const int n_tof = c.n_tof, n_planes = a.n_planes;
    const int64_t base = (int64_t)blockIdx.x * bins_per_line;
    const LineP L = a.lines[blockIdx.x];
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
            const RecGeo g = rec_geo<TOF>(a, c, L, a.planes[plane], (int)(k - (int64_t)plane * n_tof));
            CountRec it;
            it.is = (int16_t)g.is;
            it.ie = (int16_t)g.ie;
            it.pA = g.pA;
            it.pB = g.pB;
            it.zA = g.zA;
            it.zB = g.zB;
            it.me = (mult ? mult[(int64_t)blockIdx.x * n_planes + plane] : 1.f) * g.ell;
            it.y = v;
            it.add = add ? add[base + k] : 0.f;
            items[out + rank] = it;
        }
        out += total;
        __syncthreads();
    }
}

// TOF weight W(d) from the LDS table of (W_k, W_{k+1} - W_k) at its NW_TAB
// nodes, at table position pos = d / dx + NW/2 in [0, pos_max]: linear
// interpolation between the two nodes around pos (one 8-byte LDS read).
__device__ __forceinline__ float tof_weight_at(const float2 *tab, float pos) {
    const float2 t = tab[(int)pos];
    return fmaf(__builtin_amdgcn_fractf(pos), t.y, t.x);
}

// Sum over the workgroup, the same value in every thread (wave sums by
// shuffles, then the wave partials in a fixed order).
__device__ __forceinline__ float2 block_sum_all(float2 v, float2 *red) {
    for (int off = 32; off > 0; off >>= 1) {
        v.x += __shfl_xor(v.x, off, 64);
        v.y += __shfl_xor(v.y, off, 64);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float2 t = make_float2(0.f, 0.f);
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        t.x += red[w].x;
        t.y += red[w].y;
    }
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
//
// The gradient's share of a sample is -Q W: with every Q of a chunk >= 0 (the
// case whenever x >= 0 and add > 0) the sheet accumulates +Q W, whose two
// parts are both nonnegative and pack with no borrow, and the readout
// negates; otherwise it accumulates the signed shares with the borrow of a
// negative low word carried into the high one.
__device__ __forceinline__ uint32_t round_pos(float q) {
    // floor(q + 1/2) of a nonnegative q below 2^31, in one instruction
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(q));
    return (uint32_t)r;
}

__device__ __forceinline__ void deposit_pos(unsigned long long *zr, int j, float q, float f) {
    const uint32_t A = round_pos(q), B = round_pos(q * f);
    atomicAdd(&zr[j], (unsigned long long)A | ((unsigned long long)B << 32));
}

__device__ __forceinline__ void deposit_packed(unsigned long long *zr, int j, float qs, float f) {
    const int A = (int)__builtin_rintf(qs);
    const int B = (int)__builtin_rintf(qs * f);
    const unsigned long long v =
        (unsigned long long)(uint32_t)A | ((unsigned long long)(uint32_t)(B + (A >> 31)) << 32);
    atomicAdd(&zr[j], v);
}

// The two accumulators of a packed cell: the low word read as signed is A,
// and (w - A) is exactly 2^32 B (signed shares); both words unsigned
// (nonnegative shares).
template <bool SIGNED>
__device__ __forceinline__ void unpack_cell(unsigned long long w, long long &A, long long &B) {
    if (SIGNED) {
        const int lo = (int)(uint32_t)w;
        A = lo;
        B = ((long long)w - (long long)lo) >> 32;
    } else {
        A = (long long)(uint32_t)w;
        B = (long long)(w >> 32);
    }
}

// Spread the packed sheet over the two transaxial neighbours (the readout of
// the FP64 sheet in the dense kernels, after unpacking).  A line whose bound
// is not finite (a bin with ybar = 0) adds NaN to every cell it covers.
template <bool SIGNED>
__device__ __forceinline__ float packed_cell_value(const unsigned long long *Zu, int e, int zp, float inv_scale,
                                                   bool finite) {
    if (!SIGNED) {
        // nonnegative shares: B <= A in every cell (each sample's rounded
        // f q <= its rounded q), so A - B + B' < 2^32 in 32-bit arithmetic
        const unsigned long long w = Zu[e];
        const uint32_t Bp = zp > 0 ? (uint32_t)(Zu[e - 1] >> 32) : 0u;
        const uint32_t V = (uint32_t)w - (uint32_t)(w >> 32) + Bp;
        return finite ? -(float)V * inv_scale : __builtin_nanf("");
    }
    long long A, B, Ap, Bp = 0;
    unpack_cell<true>(Zu[e], A, B);
    if (zp > 0) unpack_cell<true>(Zu[e - 1], Ap, Bp);
    const long long V = A - B + Bp;
    return finite ? (float)V * inv_scale : __builtin_nanf("");
}

// Readout of the packed sheet of the line's rows of parity par (row par + 2k
// of the line in Zu row k, k < nh), spread over the two transaxial neighbours
// like the FP64 sheet of the dense kernels.  A line whose bound is not finite
// (a bin with ybar = 0) adds NaN to every cell it covers.
template <bool SIGNED>
__device__ __forceinline__ void scatter_rows_parity(const ProjArgs &a, const LineP &L, int par, int nh,
                                                    const unsigned long long *Zu, float inv_scale, bool finite,
                                                    int64_t g_off) {
    const int rz = a.rz;
    float *Gout = (L.axis ? a.G1 : a.G0) + g_off;
    const int other_stride = ((L.axis ? a.nx : a.ny) + 2 * PADA) * rz;
    if (rz <= (int)blockDim.x) {
        const SheetWalk w = sheet_walk(rz);
        if (!w.on) return;
        for (int k = w.r0; k < nh; k += w.R) {
            const float val = packed_cell_value<SIGNED>(Zu, k * rz + w.zp, w.zp, inv_scale, finite);
            if (val == 0.f) continue;
            spread_cell(Gout, sheet_row(L, L.i_lo + par + 2 * k, other_stride, rz), w.zp, rz, val);
        }
    } else {
        for (int e = threadIdx.x; e < nh * rz; e += blockDim.x) {
            const int k = e / rz;
            const int zp = e - k * rz;
            const float val = packed_cell_value<SIGNED>(Zu, e, zp, inv_scale, finite);
            if (val == 0.f) continue;
            spread_cell(Gout, sheet_row(L, L.i_lo + par + 2 * k, other_stride, rz), zp, rz, val);
        }
    }
}

// Lanes per bin of a round of n_c bins: a power of two C <= 16, doubled while
// the round's bins still fill the workgroup, so that lines with few bins (and
// the last, partial round of a long line) keep every wave busy.
__device__ __forceinline__ int lanes_per_bin(int n_c) {
    int C = 1;
    while (C < 16 && n_c * (2 * C) <= (int)blockDim.x) C *= 2;
    return C;
}

// Rows of the image sheet whose loads a thread has in flight at once.
constexpr int CNT_SHEET_ROWS = 8;

// Image sheet X of a line (rows [0, nrow), padded axial positions [0, rz)):
// the transaxial interpolation of the transposed image, as build_sheets.
__device__ __forceinline__ void build_x(const ProjArgs &a, const LineP &L, int nrow, float *X) {
    const int rz = a.rz;
    if (rz > (int)blockDim.x) {
        build_sheets<true, false>(a, L, nrow, X, nullptr);
        return;
    }
    const float *T = L.axis ? a.T1 : a.T0;
    const int other_stride = ((L.axis ? a.nx : a.ny) + 2 * PADA) * rz;
    const SheetWalk sw = sheet_walk(rz);
    if (!sw.on) return;
    for (int rb = sw.r0; rb < nrow; rb += CNT_SHEET_ROWS * sw.R) {
        float t0[CNT_SHEET_ROWS], t1[CNT_SHEET_ROWS], tf[CNT_SHEET_ROWS];
#pragma unroll
        for (int u = 0; u < CNT_SHEET_ROWS; ++u) {
            const int r = rb + u * sw.R;
            t0[u] = t1[u] = tf[u] = 0.f;
            if (r < nrow) {
                const SheetRow sr = sheet_row(L, L.i_lo + r, other_stride, rz);
                tf[u] = sr.f;
                const float *src = T + sr.base + sw.zp;
                t0[u] = src[0];
                t1[u] = src[rz];
            }
        }
#pragma unroll
        for (int u = 0; u < CNT_SHEET_ROWS; ++u) {
            const int r = rb + u * sw.R;
            if (r < nrow) X[r * rz + sw.zp] = fmaf(tf[u], t1[u] - t0[u], t0[u]);
        }
    }
}

// What phase two needs of a bin: its rows (is and ie as the two 16-bit
// halves of one word), the affine table and axial positions, and its factor Q.
struct BinB {
    uint32_t isie;
    float pA, pB, zA, zB, Q;
};

__device__ __forceinline__ BinB bin_b(const CountRec &e, float Q) {
    return {(uint32_t)(uint16_t)e.is | ((uint32_t)(uint16_t)e.ie << 16), e.pA, e.pB, e.zA, e.zB, Q};
}

// Rounds of a chunk (bins per thread) that phase two keeps in registers.
constexpr int CNT_ROUNDS = 4;
static_assert(CNT_QCAP <= CNT_ROUNDS * CNT_BLOCK, "a chunk takes at most CNT_ROUNDS rounds of one bin per thread");

// One workgroup per line with counts.  MODE M_GRAD: gradient sheets receive
// -P^T [mult y / ybar]; M_OBJ: no gradient.  Both write the workgroup's FP64
// sum of y log(y / ybar) when a.partial is set.
//
// LDS: one sheet region that holds the image sheet X (nrow x rz floats) while
// the bins are walked forward, and then the packed gradient sheet of the rows
// of one parity (ceil(nrow / 2) x rz 64-bit words, the same bytes); the TOF
// table.
// About 71 KB on the brain-sized workloads, so that two workgroups share a CU
// and one's barriers overlap the other's samples.
//
// The line's bins are taken in chunks of at most c.q_cap.  Phase one walks
// every bin of the chunk forward (ybar, the log term, Q = mult y / ybar ell).
// With M_GRAD, phase two runs once per parity of the rows (even rows, then
// odd ones, so that every bin's window splits about evenly between the two
// passes): it clears the packed sheet, adds the chunk's shares -Q W(t - t_b)
// (times the axial interpolation weights, scaled by 2^30 / sum |Q|) of the
// samples in those rows, and reads them out.  Each thread keeps what phase two needs of its bins (one per
// round of the chunk, at most CNT_ROUNDS) and their factors in registers
// between the phases.  A next chunk rebuilds X.
template <bool TOF, int MODE>
__global__ void __launch_bounds__(CNT_BLOCK) k_line_counts(ProjArgs a, CountArgs c) {
    extern __shared__ float4 smem4[];
    float *smem = reinterpret_cast<float *>(smem4);
    __shared__ float2 red[CNT_BLOCK / 64];
    constexpr bool NEED_Z = MODE == M_GRAD;
    const CountLine desc = c.desc[blockIdx.x];
    const LineP &L = desc.L;
    const int nrow = L.i_hi - L.i_lo + 1;
    const int rz = a.rz;
    float *X = smem;
    unsigned long long *Zu = reinterpret_cast<unsigned long long *>(smem);  // (X's bytes, after phase one)
    float2 *tab = reinterpret_cast<float2 *>(smem + c.sheet_floats);
    const int64_t i0 = desc.i0, i1 = desc.i0 + desc.n;
    const CountRec none{1, 0, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // no rows, no count

    if (TOF) {
        // the table's loads in flight together, eight per thread
        static_assert(NW_TAB % (8 * CNT_BLOCK) == 0, "the table load assumes 8 CNT_BLOCK divides NW_TAB");
        for (int k0 = threadIdx.x; k0 < NW_TAB; k0 += 8 * CNT_BLOCK) {
            float2 wv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) wv[u] = c.wtab[k0 + u * CNT_BLOCK];
#pragma unroll
            for (int u = 0; u < 8; ++u) tab[k0 + u * CNT_BLOCK] = wv[u];
        }
    }
    if (nrow > 0) build_x(a, L, nrow, X);
    __syncthreads();

    double kl = 0.0;
    // (a line that misses the image still has bins with counts: ybar = add there,
    // and its y log(y / add) enters the sum; its sample ranges are empty)
    for (int64_t c0 = i0; c0 < i1; c0 += c.q_cap) {
        const int64_t c1 = c0 + c.q_cap < i1 ? c0 + c.q_cap : i1;
        if (NEED_Z && c0 > i0) {
            // phase two of the previous chunk overwrote X (its last barrier
            // follows the readout)
            if (nrow > 0) build_x(a, L, nrow, X);
            __syncthreads();
        }
        // Rounds of up to one bin per thread (CNT_BLOCK threads); a round with
        // fewer bins, the chunk's last, gives each bin C lanes (consecutive
        // lanes of one wave) that take every C-th sample of its window
        const int n_c = (int)(c1 - c0);
        const int nr = (n_c + CNT_BLOCK - 1) / CNT_BLOCK;
        float qabs = 0.f, qneg = 0.f;
        // the thread's bins of the chunk's rounds (at most CNT_ROUNDS) and
        // their factors, for phase two
        BinB b0 = bin_b(none, 0.f), b1 = b0, b2 = b0, b3 = b0;
        for (int rr = 0; rr < nr; ++rr) {
            const int m = min(CNT_BLOCK, n_c - rr * CNT_BLOCK);
            const int C = lanes_per_bin(m);
            const int ch = threadIdx.x & (C - 1);
            const float fC = (float)C;
            // every lane runs every round: the forward sums are added across
            // the C lanes of a bin by shuffles
            const int k = (int)threadIdx.x / C;
            const bool act = k < m;
            const CountRec e = act ? c.items[c0 + (int64_t)rr * CNT_BLOCK + k] : none;
            // rows as floats (exact integers): no conversion per sample
            const float fis = (float)(e.is + ch), fie = (float)e.ie;
            // two samples per iteration (their LDS reads in flight together,
            // two partial sums), then the odd one; u stays in [0, rz - 1)
            // (the records' rows are cut to it)
            float s = 0.f, s1 = 0.f;
            const float *xr = X + (e.is + ch - L.i_lo) * rz;
            const int step = C * rz;
            float fi = fis;
            for (; fi + fC <= fie; fi += 2.f * fC, xr += 2 * step) {
                const float fj = fi + fC;
                const float u0 = fmaf(fi, e.zA, e.zB), u1 = fmaf(fj, e.zA, e.zB);
                const int j0 = (int)u0, j1 = (int)u1;
                const float a0 = xr[j0], b0 = xr[j0 + 1], a1 = xr[step + j1], b1 = xr[step + j1 + 1];
                const float v0 = fmaf(__builtin_amdgcn_fractf(u0), b0 - a0, a0);
                const float v1 = fmaf(__builtin_amdgcn_fractf(u1), b1 - a1, a1);
                s = TOF ? fmaf(tof_weight_at(tab, fmaf(fi, e.pA, e.pB)), v0, s) : s + v0;
                s1 = TOF ? fmaf(tof_weight_at(tab, fmaf(fj, e.pA, e.pB)), v1, s1) : s1 + v1;
            }
            if (fi <= fie) {
                const float u = fmaf(fi, e.zA, e.zB);
                const int j = (int)u;
                const float x0 = xr[j], x1 = xr[j + 1];
                const float v = fmaf(__builtin_amdgcn_fractf(u), x1 - x0, x0);
                s = TOF ? fmaf(tof_weight_at(tab, fmaf(fi, e.pA, e.pB)), v, s) : s + v;
            }
            s += s1;
            // (every lane of the bin ends with the bin's sum)
            for (int o = 1; o < C; o <<= 1) s += __shfl_xor(s, o, 64);
            const float ybar = fmaf(e.me, s, e.add);
            // (the FP64 logarithm only when the sums are wanted)
            if (a.partial && act && ch == 0) kl += (double)e.y * log((double)e.y / (double)ybar);
            if (NEED_Z) {
                const float Q = act ? e.me * e.y * __builtin_amdgcn_rcpf(ybar) : 0.f;
                if (ch == 0) {
                    qabs += fabsf(Q);
                    qneg += Q < 0.f ? 1.f : 0.f;
                }
                // (a uniform switch keeps every register index static)
                const BinB b = bin_b(e, Q);
                switch (rr) {
                    case 0: b0 = b; break;
                    case 1: b1 = b; break;
                    case 2: b2 = b; break;
                    default: b3 = b; break;
                }
            }
        }
        if (!NEED_Z) continue;  // uniform
        // (the barrier inside also ends every read of X)
        const float2 tot = block_sum_all(make_float2(qabs, qneg), red);
        const float bound = tot.x;
        const bool finite = bound < INFINITY;  // false for inf and NaN
        const bool sgn = tot.y > 0.f || c.force_signed;  // some Q < 0 (uniform)
        const float scale = finite && bound > 0.f ? 0x1p30f / bound : 0.f;
        if (nrow == 0 || (scale == 0.f && finite)) continue;  // (nothing to add; uniform)
        for (int par = 0; par < 2; ++par) {
            // the line's rows of parity par, so that every bin's window splits
            // about evenly between the two passes
            const int nh = (nrow - par + 1) >> 1;
            if (nh <= 0) break;  // (uniform)
            for (int k = threadIdx.x; k < nh * rz; k += blockDim.x) Zu[k] = 0ull;
            __syncthreads();
            if (scale > 0.f) {
                for (int q = 0; q < nr; ++q) {  // (uniform)
                    const int m = min(CNT_BLOCK, n_c - q * CNT_BLOCK);
                    const int C = lanes_per_bin(m);
                    const int ch = threadIdx.x & (C - 1);
                    const float fS = 2.f * (float)C;  // rows per step of a lane
                    BinB g;
                    switch (q) {
                        case 0: g = b0; break;
                        case 1: g = b1; break;
                        case 2: g = b2; break;
                        default: g = b3; break;
                    }
                    const float qsc = g.Q * scale;
                    const int gis = (int)(int16_t)(g.isie & 0xffffu), gie = (int)(int16_t)(g.isie >> 16);
                    // this lane's rows: the bin's first row of parity par, then
                    // every 2C-th row from 2 ch on
                    const int r0 = gis + ((gis - L.i_lo - par) & 1) + 2 * ch;
                    const float fis = (float)r0, fie = (float)gie;
                    unsigned long long *zr = Zu + ((r0 - L.i_lo - par) >> 1) * rz;
                    const int step = C * rz;  // (Zu rows per step of a lane)
                    if (!sgn) {
                        // (two samples per iteration, as forward)
                        float fi = fis;
                        for (; fi + fS <= fie; fi += 2.f * fS, zr += 2 * step) {
                            const float fj = fi + fS;
                            const float qw0 = TOF ? qsc * tof_weight_at(tab, fmaf(fi, g.pA, g.pB)) : qsc;
                            const float qw1 = TOF ? qsc * tof_weight_at(tab, fmaf(fj, g.pA, g.pB)) : qsc;
                            const float u0 = fmaf(fi, g.zA, g.zB), u1 = fmaf(fj, g.zA, g.zB);
                            deposit_pos(zr, (int)u0, qw0, __builtin_amdgcn_fractf(u0));
                            deposit_pos(zr + step, (int)u1, qw1, __builtin_amdgcn_fractf(u1));
                        }
                        if (fi <= fie) {
                            const float qw = TOF ? qsc * tof_weight_at(tab, fmaf(fi, g.pA, g.pB)) : qsc;
                            const float u = fmaf(fi, g.zA, g.zB);
                            deposit_pos(zr, (int)u, qw, __builtin_amdgcn_fractf(u));
                        }
                    } else {
                        for (float fi = fis; fi <= fie; fi += fS, zr += step) {
                            const float qw = TOF ? qsc * tof_weight_at(tab, fmaf(fi, g.pA, g.pB)) : qsc;
                            const float u = fmaf(fi, g.zA, g.zB);
                            deposit_packed(zr, (int)u, -qw, __builtin_amdgcn_fractf(u));
                        }
                    }
                }
            }
            __syncthreads();
            const int64_t g_off = (int64_t)desc.slot * c.slot_floats;
            if (sgn)
                scatter_rows_parity<true>(a, L, par, nh, Zu, finite ? 1.f / scale : 0.f, finite, g_off);
            else
                scatter_rows_parity<false>(a, L, par, nh, Zu, finite ? 1.f / scale : 0.f, finite, g_off);
            // (before the next pass clears the sheet, or the next chunk's X)
            __syncthreads();
        }
    }
    if (a.partial) block_sums(kl, kl, a.partial, false);
}

// Descriptors of a launch's lines (geometry and item ranges), one per line.
__global__ void k_counts_desc(const int *__restrict__ lines, int n, const LineP *__restrict__ geo,
                              const int64_t *__restrict__ line_off, const int *__restrict__ view_subset, int n_rad,
                              CountLine *__restrict__ desc) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int l = lines[k];
    CountLine d;
    d.L = geo[l];
    d.i0 = line_off[l];
    d.n = (int32_t)(line_off[l + 1] - line_off[l]);
    d.slot = view_subset[l / n_rad];
    desc[k] = d;
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

// LDS of the counts kernel (dynamic), in floats: the sheet region (X, or the
// packed gradient sheet of the rows of one parity), the TOF table (NW_TAB
// (W, dW) pairs), each rounded up to 16 bytes.
static size_t counts_sheet_floats(const pet_geom_s *g) {
    const size_t rz = (size_t)g->d.nz + 2 * PADZ;
    const size_t x = (size_t)g->rows_max * rz;
    const size_t zu = 2 * (((size_t)g->rows_max + 1) / 2) * rz;
    return (std::max(x, zu) + 3) & ~(size_t)3;
}

static size_t counts_tab_floats(const pet_geom_s *g) { return g->d.n_tof > 1 ? 2 * (size_t)NW_TAB : 0; }

static size_t counts_lds_base(const pet_geom_s *g) {
    return sizeof(float) * (counts_sheet_floats(g) + counts_tab_floats(g));
}

// Bins per chunk with M_GRAD: CNT_QCAP (their factors live in registers), or
// 0 if the sheet and the table (with 1 KB of static shared memory) exceed the
// LDS.
static int counts_q_cap(const pet_geom_s *g) {
    return counts_lds_base(g) + 1024 <= g->max_lds ? CNT_QCAP : 0;
}

size_t counts_lds_bytes(const pet_geom_s *g, int) { return counts_lds_base(g); }

int counts_blocks(const pet_counts_s *cs, int subset) {
    const int row = subset < 0 ? cs->n_subsets : subset;
    return (int)(cs->lines_off[row + 1] - cs->lines_off[row]);
}

// The TOF table's constants (and the TOF bin count) of a geometry.
static CountArgs count_args(const pet_geom_s *g) {
    CountArgs c{};
    c.wtab = g->wtab;
    c.nw = NW_TAB;
    c.sheet_floats = (int)counts_sheet_floats(g);
    c.tab_floats = (int)counts_tab_floats(g);
    c.n_tof = g->d.n_tof;
    c.wD = g->wD;
    c.inv_dx = (float)(NW_TAB / (2.0 * g->wD));
    c.pos0 = (float)(NW_TAB / 2);
    c.pos_max = (float)NW_TAB - 1e-3f;
    return c;
}

hipError_t launch_line_counts(pet_geom_s *g, const pet_counts_s *cs, int mode, int subset, const ProjArgs &a,
                              hipStream_t s, int64_t slot_floats) {
    const int nblk = counts_blocks(cs, subset);
    if (nblk == 0) return hipSuccess;
    if (slot_floats && (subset >= 0 || mode != M_GRAD)) return hipErrorInvalidValue;
    CountArgs c = count_args(g);
    c.slot_floats = slot_floats;
    c.items = cs->items;
    c.desc = cs->desc + cs->lines_off[subset < 0 ? cs->n_subsets : subset];
    c.q_cap = mode != M_GRAD ? (1 << 30) : (g->flags & PET_SMALL_CHUNKS) ? std::min(16, counts_q_cap(g)) : counts_q_cap(g);
    c.force_signed = (g->flags & PET_SIGNED_SHEETS) != 0;
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
    if (e == hipSuccess) e = hipMalloc(&c->items, sizeof(CountRec) * std::max<int64_t>(c->n_items, 1));
    if (e == hipSuccess) e = hipMemcpy(c->line_off, off.data(), sizeof(int64_t) * (n_lines + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess && c->n_items > 0) {
        const ProjArgs pa = geom_proj_args(g);
        const CountArgs ca = count_args(g);
        if (g->d.n_tof > 1)
            hipLaunchKernelGGL(k_counts_fill<true>, dim3(n_lines), dim3(256), 0, 0, y, y_dtype, add, mult, bpl,
                               c->line_off, pa, ca, c->items);
        else
            hipLaunchKernelGGL(k_counts_fill<false>, dim3(n_lines), dim3(256), 0, 0, y, y_dtype, add, mult, bpl,
                               c->line_off, pa, ca, c->items);
    }
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
    if (e == hipSuccess) e = hipMalloc(&c->desc, sizeof(CountLine) * std::max<size_t>(lines.size(), 1));
    // the subset of each view (the gradient-sheet slot of its lines)
    std::vector<int> vsub(g->d.n_views, 0);
    for (int q = 0; q < n; ++q)
        for (int v : g->subset_views[q]) vsub[v] = q;
    int *d_vsub = nullptr;
    if (e == hipSuccess) e = hipMalloc(&d_vsub, sizeof(int) * vsub.size());
    if (e == hipSuccess) e = hipMemcpy(d_vsub, vsub.data(), sizeof(int) * vsub.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !lines.empty()) {
        const int nl = (int)lines.size();
        hipLaunchKernelGGL(k_counts_desc, dim3((nl + 255) / 256), dim3(256), 0, 0, c->lines, nl, g->lines,
                           c->line_off, d_vsub, g->d.n_rad, c->desc);
        e = hipGetLastError();
    }
    // gradient sheets of a one-launch snapshot pass (n pairs, interiors zero
    // between snapshots), where the fused step serves the geometry
    if (e == hipSuccess && step_tile_ok(g)) {
        const int64_t stride = ((int64_t)g->t0_elems + (int64_t)g->t1_elems + 3) & ~(int64_t)3;
        e = hipMalloc(&c->slots, sizeof(float) * (size_t)(stride * n));
        if (e == hipSuccess) e = hipMemset(c->slots, 0, sizeof(float) * (size_t)(stride * n));
        if (e == hipSuccess) c->slot_floats = stride;
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (d_vsub) (void)hipFree(d_vsub);
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
    void *ptrs[] = {c->items, c->line_off, c->lines, c->desc, c->slots};
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
