// Cell-driven (gather) adjoint of the Joseph projector: pet_back with
// PET_BACK_GATHER.
//
// The scatter adjoint (proj.hip) walks the samples of every LOR of a line and
// adds each sample's two axial interpolation shares to an LDS sheet with FP64
// atomics.  Here each thread owns sheet cells (row i along the principal axis,
// interior axial cell c) instead and sums, without atomics, every share that
// lands on its cell.  A cell receives the share (1 - f) of a sample whose
// axial position u (in padded cells) has floor(u) = c and the share f of one
// with floor(u) = c - 1, i.e. from the samples with u in [c - 1, c + 1).
// Within a segment (one ring difference) the axial position at row i is
// affine in the plane's rank k, u_k = U0 + k S with S = ring pitch / vz, so
// the candidate planes follow from (c - U0) / S: about 2 / S + 1 of them,
// each checked with the exact sample position the scatter uses.  Cells of the
// axial padding are not formed: the image keeps only interior cells, and
// only samples outside the z range reach the padding, so the sum over a cell
// is the scatter's sum over the same (sample, weight) pairs.
//
// TOF: the weight of bin b at a sample at signed distance t from the LOR
// centre is the tabulated W(t - t_b) (the counts kernel's table); t depends on
// the row and the segment only, so one set of weights serves the planes of a
// segment at a cell.
//
// The finished cell values are spread over the two transaxial neighbours with
// global float atomics, as the scatter's sheet readout does.
#include "line_sheets.h"

namespace pet {
namespace {

constexpr int GATHER_BLOCK = 1024;

struct GatherArgs {
    const SegP *segs;   // plain segments in plane order
    int n_seg;
    const float2 *wtab;
    int nw;
    float wD, inv_dx, pos0, pos_max;
};

__device__ __forceinline__ float gather_weight(const float2 *tab, float d, const GatherArgs &c) {
    const float pos = __builtin_amdgcn_fmed3f(fmaf(d, c.inv_dx, c.pos0), 0.f, c.pos_max);
    const int k = (int)pos;
    const float2 t = tab[k];
    return fmaf(pos - (float)k, t.y, t.x);
}

// One workgroup per line.  LDS: per plane (zA, zB) of its axial map and its
// factor mult * ell (* sino without TOF), and the TOF weight table.
template <bool TOF>
__global__ void __launch_bounds__(GATHER_BLOCK) k_line_gather(ProjArgs a, GatherArgs ga) {
    extern __shared__ float4 smem4[];
    float *smem = reinterpret_cast<float *>(smem4);
    const int line = a.order[blockIdx.x];
    const LineP L = a.lines[line];
    const int nrow = L.i_hi - L.i_lo + 1;
    if (nrow <= 0) return;  // uniform: the whole workgroup leaves
    const int np_all = a.n_planes;
    float2 *zab = reinterpret_cast<float2 *>(smem);
    float *qf = smem + 2 * np_all;
    float2 *tab = reinterpret_cast<float2 *>(smem + ((3 * np_all + 1) & ~1));
    if (TOF)
        for (int k = threadIdx.x; k < ga.nw; k += blockDim.x) tab[k] = ga.wtab[k];
    for (int p = threadIdx.x; p < np_all; p += blockDim.x) {
        const PlaneP P = a.planes[p];
        const int64_t lor = (int64_t)line * np_all + p;
        const float ell = L.vm_um * sqrtf(L.lt2 + P.dz2);
        zab[p] = make_float2(P.zs * L.dlam, fmaf(L.lam0, P.zs, P.zb) + (float)PADZ);
        const float m = a.mult ? a.mult[lor] : 1.f;
        qf[p] = TOF ? m * ell : (a.sino ? a.sino[lor] : 1.f) * m * ell;
    }
    __syncthreads();

    const int nz = a.nz, rz = a.rz, nt = a.tof.n_tof;
    const float umax = (float)(nz + PADZ);
    float *Gout = L.axis ? a.G1 : a.G0;
    const size_t other_stride = (size_t)((L.axis ? a.nx : a.ny) + 2 * PADA) * rz;
    for (int e = threadIdx.x; e < nrow * nz; e += blockDim.x) {
        const int r = e / nz;
        const int cz = e - r * nz;
        const int i = L.i_lo + r;
        const float fi = (float)i;
        const int cp = cz + PADZ;  // padded axial cell
        const float cpf = (float)cp;
        float acc = 0.f;
        for (int sgi = 0; sgi < ga.n_seg; ++sgi) {
            const SegP sg = ga.segs[sgi];
            const float2 ab0 = zab[sg.p0];
            const float u0 = fmaf(fi, ab0.x, ab0.y);
            int klo = 0, khi = sg.np - 1;
            if (sg.np > 1) {
                const float2 ab1 = zab[sg.p0 + sg.np - 1];
                const float S = (fmaf(fi, ab1.x, ab1.y) - u0) / (float)(sg.np - 1);
                // planes with u in [c - 1, c + 1), one rank of margin each side
                const float ka = (cpf - 1.f - u0) / S, kb = (cpf + 1.f - u0) / S;
                // (clamped to [-1, np] before the conversion)
                const float lo = fminf(fmaxf(floorf(fminf(ka, kb)) - 1.f, -1.f), (float)sg.np);
                const float hi = fmaxf(fminf(ceilf(fmaxf(ka, kb)) + 1.f, (float)sg.np), -1.f);
                klo = max(klo, (int)lo);
                khi = min(khi, (int)hi);
            }
            if (klo > khi) continue;
            float w[WS_MAX];
            int b_lo = 0, nb = 0;
            if (TOF) {
                // weights of the bins this row's sample sees (same for every
                // plane of the segment)
                const float len = sqrtf(L.lt2 + sg.dz2);
                const float t = (fmaf(fi, L.dlam, L.lam0) - 0.5f) * len;
                const float tb0 = a.tof.tb[0], bw = 2.f * a.tof.half_bin;
                b_lo = max(0, (int)ceilf((t - ga.wD - tb0) / bw));
                const int b_hi = min(nt - 1, (int)floorf((t + ga.wD - tb0) / bw));
                nb = min(b_hi - b_lo + 1, WS_MAX);
#pragma unroll
                for (int j = 0; j < WS_MAX; ++j)
                    w[j] = j < nb ? gather_weight(tab, t - a.tof.tb[min(b_lo + j, nt - 1)], ga) : 0.f;
            }
            for (int k = klo; k <= khi; ++k) {
                const int p = sg.p0 + k;
                const float2 ab = zab[p];
                const float u = __builtin_amdgcn_fmed3f(fmaf(fi, ab.x, ab.y), 0.f, umax);
                const int j = (int)u;
                const float f = __builtin_amdgcn_fractf(u);
                const float wz = j == cp ? 1.f - f : (j + 1 == cp ? f : 0.f);
                if (wz == 0.f) continue;
                float q = qf[p];
                if (TOF) {
                    const float *sr = a.sino ? a.sino + ((int64_t)line * np_all + p) * nt + b_lo : nullptr;
                    float sb = 0.f;
#pragma unroll
                    for (int jb = 0; jb < WS_MAX; ++jb)
                        if (jb < nb) sb = fmaf(w[jb], sr ? sr[min(jb, nb - 1)] : 1.f, sb);
                    q *= sb;
                }
                acc = fmaf(wz, q, acc);
            }
        }
        if (acc == 0.f) continue;
        // transaxial spread, as the scatter's sheet readout
        const float xa = fmaf(fi, L.dxa, L.xa0);
        const float jf = floorf(xa);
        const float fa = xa - jf;
        const size_t base = (size_t)i * other_stride + (size_t)((int)jf + PADA) * rz + cp;
        const float a1 = acc * fa;
        atomicAdd(&Gout[base], acc - a1);
        atomicAdd(&Gout[base + rz], a1);
    }
}

template <bool TOF>
void set_gather_lds(size_t need) {
    static size_t granted = 64 * 1024;
    if (need <= granted) return;
    if (hipFuncSetAttribute((const void *)k_line_gather<TOF>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)need) == hipSuccess)
        granted = need;
    (void)hipGetLastError();
}

}  // namespace

size_t gather_lds_bytes(const pet_geom_s *g) {
    const size_t planes = ((size_t)3 * g->n_planes + 1) & ~(size_t)1;
    return planes * sizeof(float) + (g->d.n_tof > 1 ? sizeof(float2) * NW_TAB : 0);
}

hipError_t launch_line_gather(pet_geom_s *g, int subset, const ProjArgs &a, hipStream_t s) {
    const int nblk = n_line_blocks(g, subset);
    if (nblk == 0) return hipSuccess;
    GatherArgs ga{};
    ga.segs = g->gsegs;
    ga.n_seg = g->n_gseg;
    ga.wtab = g->wtab;
    ga.nw = NW_TAB;
    ga.wD = g->wD;
    ga.inv_dx = g->d.n_tof > 1 ? (float)(NW_TAB / (2.0 * g->wD)) : 0.f;
    ga.pos0 = (float)(NW_TAB / 2);
    ga.pos_max = (float)NW_TAB - 1e-3f;
    const size_t lds = gather_lds_bytes(g);
    hipEvent_t e1 = nullptr;
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
        e1 = ev.second;
        g->prof_events[PROF_GATHER].push_back(ev);
        e = hipEventRecord(ev.first, s);
    }
    if (e == hipSuccess) {
        if (g->d.n_tof > 1) {
            set_gather_lds<true>(lds);
            hipLaunchKernelGGL(k_line_gather<true>, dim3(nblk), dim3(GATHER_BLOCK), lds, s, a, ga);
        } else {
            set_gather_lds<false>(lds);
            hipLaunchKernelGGL(k_line_gather<false>, dim3(nblk), dim3(GATHER_BLOCK), lds, s, a, ga);
        }
        e = hipGetLastError();
    }
    if (e == hipSuccess && e1) e = hipEventRecord(e1, s);
    return e;
}

}  // namespace pet
