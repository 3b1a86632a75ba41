// Host-side geometry (FP64) for the gfx950 PET library: LOR endpoints from the
// scanner description, per-line Joseph sampling parameters, per-plane axial
// parameters, TOF interval table and TOF weight table, plus the scratch arena.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "pet_internal.h"

using namespace pet;

namespace {

struct Plane {
    int r1, r2, seg;
};

std::vector<Plane> make_planes(const pet_geom_desc &d) {
    std::vector<Plane> out;
    if (d.kind == PET_SCANNER_PARALLEL2D) {
        out.push_back({0, 0, 0});
        return out;
    }
    std::vector<int> segs{0};
    for (int k = 1; k <= d.max_ring_diff; ++k) {
        segs.push_back(-k);
        segs.push_back(k);
    }
    for (size_t si = 0; si < segs.size(); ++si) {
        int dd = segs[si];
        for (int r1 = std::max(0, -dd); r1 < std::min(d.n_rings, d.n_rings - dd); ++r1)
            out.push_back({r1, r1 + dd, (int)si});
    }
    return out;
}

pet_status validate(const pet_geom_desc &d) {
    if (d.kind != PET_SCANNER_PARALLEL2D && d.kind != PET_SCANNER_CYLINDER)
        return fail(PET_E_ARG, "pet_geom_create: unknown scanner kind");
    if (d.nx < 1 || d.ny < 1 || d.nz < 1 || !(d.vx > 0) || !(d.vy > 0) || !(d.vz > 0))
        return fail(PET_E_ARG, "pet_geom_create: image sizes and voxel sizes must be positive");
    if (d.nz > 400) return fail(PET_E_ARG, "pet_geom_create: at most 400 axial voxels");
    if ((int64_t)d.nx * d.ny * d.nz >= ((int64_t)1 << 31)) return fail(PET_E_ARG, "pet_geom_create: too many voxels");
    if (d.nx > 32000 || d.ny > 32000 || d.nz > 32000)
        return fail(PET_E_ARG, "pet_geom_create: image dimension too large");
    if (d.n_views < 1 || d.n_rad < 1) return fail(PET_E_ARG, "pet_geom_create: n_views and n_rad must be >= 1");
    if (d.n_subsets < 1 || d.n_subsets > d.n_views)
        return fail(PET_E_ARG, "pet_geom_create: need 1 <= n_subsets <= n_views");
    if (d.n_tof < 1 || d.n_tof > NT_MAX) return fail(PET_E_ARG, "pet_geom_create: n_tof must be in [1, 32]");
    if (d.n_tof > 1 && (!(d.tof_bin_mm > 0) || !(d.tof_sigma_mm > 0) || !(d.tof_nsigma > 0)))
        return fail(PET_E_ARG, "pet_geom_create: TOF needs tof_bin_mm, tof_sigma_mm, tof_nsigma > 0");
    if (d.kind == PET_SCANNER_CYLINDER) {
        if (!(d.radius_mm > 0) || d.n_crystals != 2 * d.n_views || d.n_rings < 1 || !(d.ring_pitch_mm > 0) ||
            d.max_ring_diff < 0 || d.max_ring_diff >= d.n_rings)
            return fail(PET_E_ARG, "pet_geom_create: inconsistent cylinder description "
                                   "(need radius > 0, n_crystals = 2 n_views, 0 <= max_ring_diff < n_rings)");
        if (d.n_rad > d.n_crystals) return fail(PET_E_ARG, "pet_geom_create: n_rad > n_crystals");
    } else {
        if (d.nz != 1) return fail(PET_E_ARG, "pet_geom_create: 2D parallel-beam geometry needs nz = 1");
        if (!(d.rad_spacing_mm > 0) || !(d.half_length_mm > 0))
            return fail(PET_E_ARG, "pet_geom_create: parallel-beam needs rad_spacing_mm, half_length_mm > 0");
    }
    if (!(d.psf_fwhm_mm >= 0) || !std::isfinite(d.psf_fwhm_mm))
        return fail(PET_E_ARG, "pet_geom_create: psf_fwhm_mm must be finite and >= 0");
    return PET_OK;
}

// Separable Gaussian of the resolution model, one axis: sigma in voxels,
// radius floor(4 sigma + 1/2), weights normalised to sum 1 over -r..r.
bool make_psf_axis(double sigma_vox, int axis, PsfAxis &k) {
    const int r = (int)(4.0 * sigma_vox + 0.5);
    if (r > PSF_RMAX) return false;
    double w[PSF_RMAX + 1], sum = 0.0;
    for (int i = 0; i <= r; ++i) {
        w[i] = std::exp(-0.5 * (double)i * i / (sigma_vox * sigma_vox));
        sum += i == 0 ? w[i] : 2.0 * w[i];
    }
    k.r = r;
    k.axis = axis;
    for (int i = 0; i <= PSF_RMAX; ++i) k.w[i] = i <= r ? (float)(w[i] / sum) : 0.f;
    return true;
}

}  // namespace

extern "C" pet_status pet_geom_create(const pet_geom_desc *desc, pet_geom *out) {
    if (!desc || !out) return fail(PET_E_ARG, "pet_geom_create: null argument");
    const pet_geom_desc &d = *desc;
    pet_status st = validate(d);
    if (st != PET_OK) return st;

    pet_geom_s *g = new (std::nothrow) pet_geom_s();
    if (!g) return fail(PET_E_OOM, "pet_geom_create: host allocation failed");
    g->d = d;
    if (d.psf_fwhm_mm > 0) {
        const double sig = d.psf_fwhm_mm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
        const double vox[3] = {d.vx, d.vy, d.vz};
        g->psf_passes = d.nz > 1 ? 3 : 2;
        for (int a = 0; a < g->psf_passes; ++a)
            if (!make_psf_axis(sig / vox[a], a, g->psf[a])) {
                delete g;
                return fail(PET_E_ARG, "pet_geom_create: resolution kernel wider than 16 voxels");
            }
    }
    if (hipGetDevice(&g->device) != hipSuccess) {
        delete g;
        return fail(PET_E_HIP, "pet_geom_create: no HIP device");
    }
    std::vector<Plane> planes = make_planes(d);
    g->n_planes = (int)planes.size();
    g->n_vox = (int64_t)d.nx * d.ny * d.nz;
    for (auto &p : planes) g->seg_of_plane.push_back(p.seg);

    const int N[3] = {d.nx, d.ny, d.nz};
    const double V[3] = {d.vx, d.vy, d.vz};
    double O[3];
    for (int a = 0; a < 3; ++a) O[a] = -0.5 * (N[a] - 1) * V[a];

    // axial table
    std::vector<double> z1(planes.size()), z2(planes.size());
    double max_dz = 0.0;
    for (size_t p = 0; p < planes.size(); ++p) {
        if (d.kind == PET_SCANNER_CYLINDER) {
            z1[p] = (planes[p].r1 - 0.5 * (d.n_rings - 1)) * d.ring_pitch_mm;
            z2[p] = (planes[p].r2 - 0.5 * (d.n_rings - 1)) * d.ring_pitch_mm;
        } else {
            z1[p] = z2[p] = 0.0;
        }
        max_dz = std::max(max_dz, std::fabs(z2[p] - z1[p]));
    }
    std::vector<PlaneP> hplanes(planes.size());
    for (size_t p = 0; p < planes.size(); ++p) {
        hplanes[p].zb = (float)((z1[p] - O[2]) / V[2]);
        hplanes[p].zs = (float)((z2[p] - z1[p]) / V[2]);
        hplanes[p].dz2 = (float)((z2[p] - z1[p]) * (z2[p] - z1[p]));
        hplanes[p].seg = planes[p].seg;
    }

    // line table
    const int nl = d.n_views * d.n_rad;
    std::vector<LineP> hlines(nl);
    int rows_max = 0;
    for (int v = 0; v < d.n_views; ++v) {
        double phi = M_PI * v / d.n_views;
        double nx_ = std::cos(phi), ny_ = std::sin(phi), tx = -std::sin(phi), ty = std::cos(phi);
        for (int k = 0; k < d.n_rad; ++k) {
            double s, h;
            if (d.kind == PET_SCANNER_CYLINDER) {
                s = d.radius_mm * std::sin(M_PI * (k - 0.5 * (d.n_rad - 1)) / d.n_crystals);
                h = std::sqrt(d.radius_mm * d.radius_mm - s * s);
            } else {
                s = (k - 0.5 * (d.n_rad - 1)) * d.rad_spacing_mm;
                h = d.half_length_mm;
            }
            double p1[2] = {s * nx_ - h * tx, s * ny_ - h * ty};
            double u[2] = {2 * h * tx, 2 * h * ty};
            double rx = std::fabs(u[0]) / V[0], ry = std::fabs(u[1]) / V[1];
            int m = (ry > rx * (1.0 + 1e-9)) ? 1 : 0;
            double best = std::max(rx, ry);
            if (max_dz / V[2] > best * (1.0 + 1e-9)) {
                delete g;
                return fail(PET_E_ARG, "pet_geom_create: some LOR has z as principal axis (unsupported)");
            }
            int a = 1 - m;
            LineP L{};
            double lam0 = (O[m] - p1[m]) / u[m];
            double dlam = V[m] / u[m];
            double xa0 = (p1[a] + lam0 * u[a] - O[a]) / V[a];
            double dxa = dlam * u[a] / V[a];
            double lo_c, hi_c;
            if (dxa == 0.0) {
                bool in = xa0 >= -1.5 && xa0 <= N[a] + 0.5;
                lo_c = in ? 0 : 1;
                hi_c = in ? N[m] - 1 : 0;
            } else {
                double ia = (-1.5 - xa0) / dxa, ib = (N[a] + 0.5 - xa0) / dxa;
                lo_c = std::ceil(std::min(ia, ib));
                hi_c = std::floor(std::max(ia, ib));
            }
            // clamp in floating point before converting (near-axis-aligned lines
            // that miss the grid give bounds far outside the int range)
            lo_c = std::max(0.0, lo_c);
            hi_c = std::min((double)N[m] - 1, hi_c);
            int i_lo = 1, i_hi = 0;
            if (lo_c <= hi_c) {
                i_lo = (int)lo_c;
                i_hi = (int)hi_c;
                double l_a = lam0 + i_lo * dlam, l_b = lam0 + i_hi * dlam;
                if (std::min(l_a, l_b) < 0.0 || std::max(l_a, l_b) > 1.0) {
                    delete g;
                    return fail(PET_E_ARG, "pet_geom_create: LOR endpoints lie inside the padded image box");
                }
                rows_max = std::max(rows_max, i_hi - i_lo + 1);
            }
            L.lam0 = (float)lam0;
            L.dlam = (float)dlam;
            L.xa0 = (float)xa0;
            L.dxa = (float)dxa;
            L.vm_um = (float)(V[m] / std::fabs(u[m]));
            L.lt2 = (float)(u[0] * u[0] + u[1] * u[1]);
            L.i_lo = (int16_t)i_lo;
            L.i_hi = (int16_t)i_hi;
            L.axis = m;
            hlines[(size_t)v * d.n_rad + k] = L;
        }
    }

    // subsets: views v = i (mod n)
    g->subset_views.resize(d.n_subsets);
    for (int v = 0; v < d.n_views; ++v) g->subset_views[v % d.n_subsets].push_back(v);
    g->max_views = (int)g->subset_views[0].size();
    g->views_stride = d.n_views;
    std::vector<int> hviews((size_t)(d.n_subsets + 1) * d.n_views, 0);
    for (int i = 0; i < d.n_subsets; ++i)
        for (size_t j = 0; j < g->subset_views[i].size(); ++j) hviews[(size_t)i * d.n_views + j] = g->subset_views[i][j];
    for (int v = 0; v < d.n_views; ++v) hviews[(size_t)d.n_subsets * d.n_views + v] = v;
    // line launches: the lines of each subset (then of all views),
    // longest first (a line's work grows with its rows), so that the last
    // workgroups of a launch run short lines
    std::vector<int> horder;
    horder.reserve(2 * (size_t)d.n_views * d.n_rad);
    for (int row = 0; row <= d.n_subsets; ++row) {
        g->order_off.push_back((int64_t)horder.size());
        const size_t start = horder.size();
        const int nvr = row < d.n_subsets ? (int)g->subset_views[row].size() : d.n_views;
        for (int j = 0; j < nvr; ++j)
            for (int k = 0; k < d.n_rad; ++k) horder.push_back(hviews[(size_t)row * d.n_views + j] * d.n_rad + k);
        auto rows_of = [&](int l) { return std::max(0, hlines[l].i_hi - hlines[l].i_lo + 1); };
        std::stable_sort(horder.begin() + start, horder.end(), [&](int p, int q) { return rows_of(p) > rows_of(q); });
    }

    // TOF tables
    TofTable &T = g->tof;
    T.n_tof = d.n_tof;
    if (d.n_tof > 1) {
        double cut = 0.5 * d.tof_bin_mm + d.tof_nsigma * d.tof_sigma_mm;  // support of a bin's weight
        std::vector<double> tb(d.n_tof), edges;
        for (int b = 0; b < d.n_tof; ++b) {
            tb[b] = (b - 0.5 * (d.n_tof - 1)) * d.tof_bin_mm;
            T.tb[b] = (float)tb[b];
            edges.push_back(tb[b] - cut);
            edges.push_back(tb[b] + cut);
        }
        std::sort(edges.begin(), edges.end());
        std::vector<double> ue;
        for (double e : edges)
            if (ue.empty() || e - ue.back() > 1e-9 * (1.0 + std::fabs(e))) ue.push_back(e);
        T.n_int = (int)ue.size() - 1;
        for (size_t e = 0; e < ue.size(); ++e) T.edge[e] = (float)ue[e];
        for (int s = 0; s < T.n_int; ++s) {
            double mid = 0.5 * (ue[s] + ue[s + 1]);
            int bf = -1, bl = -1;
            for (int b = 0; b < d.n_tof; ++b)
                if (std::fabs(mid - tb[b]) <= cut) {
                    if (bf < 0) bf = b;
                    bl = b;
                }
            if (bf < 0) {
                bf = 0;
                bl = -1;
            }
            T.bf[s] = bf;
            T.na[s] = bl - bf + 1;
            if (T.na[s] > 8) {
                delete g;
                return fail(PET_E_ARG, "pet_geom_create: more than 8 TOF bins overlap at one point");
            }
        }
        T.half_bin = (float)(0.5 * d.tof_bin_mm);
        T.inv_sqrt2_sigma = (float)(1.0 / (std::sqrt(2.0) * d.tof_sigma_mm));
        T.erf_clamp = (float)(d.tof_nsigma / std::sqrt(2.0));
    } else {
        T.n_int = 0;
    }

    // segments (contiguous plane ranges of equal ring difference)
    std::vector<SegP> hsegs;
    for (size_t p = 0; p < planes.size(); ++p) {
        if (hsegs.empty() || planes[p].seg != planes[p - 1].seg) hsegs.push_back({(int)p, 0, hplanes[p].dz2, 0});
        hsegs.back().np++;
    }
    // the plain segment list in plane order (the gather adjoint walks it)
    const std::vector<SegP> gsegs = hsegs;
    if (d.n_tof > 1) {
        // segments -k and +k (adjacent in the plane order) have the same
        // oblique length and so the same TOF weight table: one segment wave
        // takes both when their planes fit in its 64 lanes
        std::vector<SegP> merged;
        for (const SegP &sg : hsegs) {
            const int k = std::abs(planes[sg.p0].r2 - planes[sg.p0].r1);
            if (!merged.empty()) {
                SegP &m = merged.back();
                // (the last group must still be a single segment)
                if (k > 0 && std::abs(planes[m.p0].r2 - planes[m.p0].r1) == k && m.p0 + m.np == sg.p0 &&
                    planes[m.p0].seg == planes[m.p0 + m.np - 1].seg && m.np + sg.np <= 64) {
                    m.np += sg.np;
                    continue;
                }
            }
            merged.push_back(sg);
        }
        hsegs.swap(merged);
    }
    g->n_seg = (int)hsegs.size();
    g->rows_max = rows_max;
    // non-TOF: one thread per plane, in as many waves as the planes need (up to
    // 16; more resident waves hide the LDS latency of the sample loop)
    g->nt_threads = std::min(NT_BLOCK, std::max(64, (g->n_planes + 63) / 64 * 64));
    if (d.n_tof > 1) {
        for (auto &sg : hsegs)
            if (sg.np > 64) {
                delete g;
                return fail(PET_E_ARG, "pet_geom_create: TOF needs at most 64 planes per segment (one wave)");
            }
        int ws = 1;
        for (int s = 0; s < T.n_int; ++s) ws = std::max(ws, T.na[s]);
        g->tof_ws = ws;
        // as many segment waves as the LDS holds (up to 16): the line body
        // waits on LDS latency, and more resident waves hide it better than an
        // even number of segments per wave saves
        g->tof_waves = std::min(g->n_seg, TOF_MAX_WAVES);
    }

    // LDS need of the line kernels: image sheet (float) + gradient sheet
    // (double) + per-wave TOF tables (weights [rows][4] + [rows][ws - 4] +
    // interval cuts).  Fewer TOF waves are used if the tables do not fit.
    int rz = d.nz + 2 * PADZ;
    size_t sheet = ((size_t)rows_max * rz + 3) & ~(size_t)3;
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, g->device) != hipSuccess) max_lds = 0;
    if (max_lds <= 0) max_lds = 64 * 1024;
    g->max_lds = (size_t)max_lds;
    size_t need = 3 * sheet * sizeof(float);
    if (d.n_tof > 1) {
        int e1 = g->tof_ws > 4 ? g->tof_ws - 4 : 0;
        size_t per_wave = (((size_t)rows_max * (4 + e1) + tof_cuts_pad(g->tof.n_int) + 3) & ~(size_t)3) * sizeof(float);
        if (need + per_wave <= (size_t)max_lds) {
            int fit = (int)(((size_t)max_lds - need) / per_wave);
            if (fit < g->tof_waves) g->tof_waves = fit;
        } else {
            g->tof_waves = 1;
        }
        need += (size_t)g->tof_waves * per_wave;
    }
    g->lds_bytes = need;
    // Segment order of the TOF line kernel, whose wave w takes entries w,
    // w + W, w + 2W, ... (W waves): the two halves -k and +k of a pair of
    // single segments have the same oblique length and so the same weight
    // table, and go to consecutive rounds of one wave, which then fills the
    // table once (both carry the same squared axial extent).  The other
    // entries keep their relative order.
    if (d.n_tof > 1 && g->tof_waves > 1) {
        const int W = g->tof_waves, ns = (int)hsegs.size();
        auto ring_k = [&](const SegP &sg) { return std::abs(planes[sg.p0].r2 - planes[sg.p0].r1); };
        auto single = [&](const SegP &sg) { return planes[sg.p0].seg == planes[sg.p0 + sg.np - 1].seg; };
        std::vector<int> cap(W);
        for (int w = 0; w < W; ++w) cap[w] = ns / W + (w < ns % W ? 1 : 0);
        std::vector<std::vector<int>> lists(W);
        std::vector<int> rest;
        int w = 0;
        for (int i = 0; i < ns; ++i) {
            const bool pair = i + 1 < ns && single(hsegs[i]) && single(hsegs[i + 1]) && ring_k(hsegs[i]) > 0 &&
                              ring_k(hsegs[i]) == ring_k(hsegs[i + 1]);
            if (!pair) {
                rest.push_back(i);
                continue;
            }
            hsegs[i + 1].dz2 = hsegs[i].dz2;
            int tries = 0;
            while (tries < W && (int)lists[w].size() + 2 > cap[w]) {
                w = (w + 1) % W;
                ++tries;
            }
            if (tries < W) {
                lists[w].push_back(i);
                lists[w].push_back(i + 1);
                w = (w + 1) % W;
            } else {
                rest.push_back(i);
                rest.push_back(i + 1);
            }
            ++i;
        }
        // the remaining entries fill the free slots in position order
        size_t next = 0;
        for (int r = 0; r <= ns / W; ++r)
            for (int v = 0; v < W; ++v)
                if (r < cap[v] && r >= (int)lists[v].size()) lists[v].push_back(rest[next++]);
        std::vector<SegP> ordered(ns);
        for (int v = 0; v < W; ++v)
            for (size_t r = 0; r < lists[v].size(); ++r) ordered[r * W + v] = hsegs[lists[v][r]];
        hsegs.swap(ordered);
    }
    if (g->lds_bytes > (size_t)max_lds) {
        delete g;
        return fail(PET_E_ARG, "pet_geom_create: image too large for the LDS sheets of the line kernels (" +
                                   std::to_string(g->lds_bytes) + " > " + std::to_string(max_lds) + " bytes)");
    }

    // device allocations
    auto alloc = [&](void **p, size_t bytes) { return hipMalloc(p, bytes == 0 ? 16 : bytes) == hipSuccess; };
    g->t0_elems = (size_t)d.nx * (d.ny + 2 * PADA) * rz;
    g->t1_elems = (size_t)d.ny * (d.nx + 2 * PADA) * rz;
    if (std::max(g->t0_elems, g->t1_elems) >= (size_t)INT32_MAX) {
        delete g;
        return fail(PET_E_ARG, "pet_geom_create: image too large for the 32-bit offsets of the line kernels");
    }
    // line-kernel partials (2 per line) or two per image block (BB dots)
    g->n_partial = std::max<size_t>(2 * (size_t)nl, 2 * (size_t)((g->n_vox + IMG_BLOCK - 1) / IMG_BLOCK)) + 64;
    bool ok = alloc((void **)&g->lines, sizeof(LineP) * nl) && alloc((void **)&g->planes, sizeof(PlaneP) * planes.size()) &&
              alloc((void **)&g->segs, sizeof(SegP) * hsegs.size()) &&
              alloc((void **)&g->gsegs, sizeof(SegP) * gsegs.size()) &&
              alloc((void **)&g->views_dev, sizeof(int) * hviews.size()) &&
              alloc((void **)&g->line_order, sizeof(int) * horder.size()) &&
              alloc((void **)&g->T0, sizeof(float) * g->t0_elems) && alloc((void **)&g->T1, sizeof(float) * g->t1_elems) &&
              alloc((void **)&g->G0, sizeof(float) * g->t0_elems) && alloc((void **)&g->G1, sizeof(float) * g->t1_elems) &&
              alloc((void **)&g->g, sizeof(float) * g->n_vox) && alloc((void **)&g->xtmp, sizeof(float) * g->n_vox) &&
              alloc((void **)&g->grad, sizeof(float) * g->n_vox) && alloc((void **)&g->hess, sizeof(float) * g->n_vox) &&
              alloc((void **)&g->num, sizeof(float) * g->n_vox) && alloc((void **)&g->sensi, sizeof(float) * g->n_vox) &&
              alloc((void **)&g->partial, sizeof(double) * g->n_partial) && alloc((void **)&g->dscratch, sizeof(double) * 16) &&
              alloc((void **)&g->check_counts, sizeof(unsigned) * CHECK_SLOTS) &&
              alloc((void **)&g->fscratch, sizeof(float) * 16);
    if (ok && g->psf_passes)
        ok = alloc((void **)&g->psf_a, sizeof(float) * g->n_vox) && alloc((void **)&g->psf_b, sizeof(float) * g->n_vox);
    if (!ok) {
        pet_geom_destroy(g);
        return fail(PET_E_OOM, "pet_geom_create: device allocation failed");
    }
    hipError_t e = hipMemcpy(g->lines, hlines.data(), sizeof(LineP) * nl, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(g->planes, hplanes.data(), sizeof(PlaneP) * planes.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(g->segs, hsegs.data(), sizeof(SegP) * hsegs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(g->gsegs, gsegs.data(), sizeof(SegP) * gsegs.size(), hipMemcpyHostToDevice);
    g->n_gseg = (int)gsegs.size();
    if (e == hipSuccess) e = hipMemcpy(g->views_dev, hviews.data(), sizeof(int) * hviews.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(g->line_order, horder.data(), sizeof(int) * horder.size(), hipMemcpyHostToDevice);
    // TOF weight table (FP64 nodes): W at NW_TAB + 1 nodes over |d| <= D = bin/2 + nsig sigma
    if (e == hipSuccess && d.n_tof > 1) {
        const double h = 0.5 * d.tof_bin_mm, sig = d.tof_sigma_mm, cl = d.tof_nsigma / std::sqrt(2.0);
        const double D = h + d.tof_nsigma * sig;
        g->wD = (float)D;
        auto E = [&](double u) { return std::erf(std::min(std::max(u / (std::sqrt(2.0) * sig), -cl), cl)); };
        std::vector<double> W(NW_TAB + 1);
        for (int k = 0; k <= NW_TAB; ++k) {
            const double dd = -D + 2.0 * D * k / NW_TAB;
            W[k] = k == 0 || k == NW_TAB ? 0.0 : 0.5 * (E(h - dd) - E(-h - dd));
        }
        std::vector<float2> tab(NW_TAB);
        for (int k = 0; k < NW_TAB; ++k) tab[k] = make_float2((float)W[k], (float)(W[k + 1] - W[k]));
        e = hipMalloc(&g->wtab, sizeof(float2) * NW_TAB);
        if (e == hipSuccess) e = hipMemcpy(g->wtab, tab.data(), sizeof(float2) * NW_TAB, hipMemcpyHostToDevice);
        std::vector<float> tabf(NW_TAB + 1);
        for (int k = 0; k <= NW_TAB; ++k) tabf[k] = (float)W[k];
        if (e == hipSuccess) e = hipMalloc(&g->wtabf, sizeof(float) * (NW_TAB + 1));
        if (e == hipSuccess)
            e = hipMemcpy(g->wtabf, tabf.data(), sizeof(float) * (NW_TAB + 1), hipMemcpyHostToDevice);
    }
    // padded sheet borders must be zero once; interiors are rewritten per use
    if (e == hipSuccess) e = hipMemset(g->T0, 0, sizeof(float) * g->t0_elems);
    if (e == hipSuccess) e = hipMemset(g->T1, 0, sizeof(float) * g->t1_elems);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        pet_geom_destroy(g);
        return hip_check(e, "pet_geom_create");
    }
    // set-up of the allocation-free entry point on this device (its scratch
    // array's address; a failure is reported by that entry point itself)
    void *scratch_addr = nullptr;
    (void)noalloc_scratch(g->device, &scratch_addr);
    *out = g;
    return PET_OK;
}

extern "C" pet_status pet_geom_destroy(pet_geom g) {
    if (!g) return PET_OK;
    (void)hipDeviceSynchronize();  // best effort: destruction goes on whatever it returns
    for (auto &v : g->prof_events)
        for (auto &e : v) g->prof_pool.push_back(e);
    for (auto &e : g->prof_pool) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    void *ptrs[] = {g->lines, g->planes, g->segs, g->views_dev, g->line_order, g->T0, g->T1, g->G0, g->G1, g->g, g->xtmp,
                    g->grad, g->hess, g->num, g->sensi, g->partial, g->dscratch, g->fscratch, g->psf_a, g->psf_b,
                    g->check_counts, g->wtab, g->wtabf, g->gsegs};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete g;
    return PET_OK;
}

extern "C" pet_status pet_geom_info(pet_geom g, int subset, int64_t *n_bins, int64_t *n_lors, int64_t *n_vox) {
    if (!g) return fail(PET_E_ARG, "pet_geom_info: null handle");
    if (subset < -1 || subset >= g->d.n_subsets) return fail(PET_E_ARG, "pet_geom_info: subset out of range");
    int64_t nv = subset < 0 ? g->d.n_views : (int64_t)g->subset_views[subset].size();
    int64_t lors = nv * g->d.n_rad * g->n_planes;
    if (n_lors) *n_lors = lors;
    if (n_bins) *n_bins = lors * g->d.n_tof;
    if (n_vox) *n_vox = g->n_vox;
    return PET_OK;
}
