// Allocation-free subset gradient (pet_subset_grad_noalloc).
//
// pet_subset_grad runs in the geometry handle's own work buffers.  This entry
// point runs the same kernels with every work buffer (the transposed image and
// gradient sheets, the per-line FP64 partial sums and, with a resolution model,
// two image-sized buffers) carved out of one file-scope device array instead,
// so a call allocates nothing.  Each device holds its own copy of the array, at
// its own address, from the moment the library's code object is loaded on it
// until the process ends.  Host code never uses the array's name as an
// address: the device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and kept in `g_scratch`.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "pet_internal.h"

namespace pet {
namespace {

constexpr size_t SCRATCH_BYTES = PET_NOALLOC_SCRATCH_BYTES;
constexpr size_t ALIGN = 256;

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[MAX_DEVICES];  // device address of `scratch` on device d (null until looked up)

size_t round_up(size_t n) { return (n + ALIGN - 1) / ALIGN * ALIGN; }

// Bytes of scratch one call on `subset` of geometry g needs, and the layout.
struct Layout {
    size_t t0, t1, g0, g1, psf_a, psf_b, partial, counts, total;
};
Layout layout_of(const pet_geom_s *g, int subset) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += round_up(bytes);
        return at;
    };
    L.t0 = take(sizeof(float) * g->t0_elems);
    L.t1 = take(sizeof(float) * g->t1_elems);
    L.g0 = take(sizeof(float) * g->t0_elems);
    L.g1 = take(sizeof(float) * g->t1_elems);
    L.psf_a = g->psf_passes ? take(sizeof(float) * (size_t)g->n_vox) : 0;
    L.psf_b = g->psf_passes ? take(sizeof(float) * (size_t)g->n_vox) : 0;
    L.partial = take(sizeof(double) * (size_t)n_line_blocks(g, subset));
    L.counts = take(sizeof(unsigned) * CHECK_SLOTS);
    L.total = off;
    return L;
}

}  // namespace

// Device address of this device's copy of the scratch array; looked up on the
// first call for the device, with that device current.
pet_status noalloc_scratch(int device, void **out) {
    if (device < 0 || device >= MAX_DEVICES) return fail(PET_E_ARG, "noalloc scratch: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != device) e = hipSetDevice(device);
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return hip_check(e, "noalloc scratch: hipGetSymbolAddress");
        if (!p) return fail(PET_E_HIP, "noalloc scratch: hipGetSymbolAddress returned no address");
        g_scratch[device] = p;
    }
    *out = g_scratch[device];
    return PET_OK;
}

}  // namespace pet

using namespace pet;

extern "C" pet_status pet_subset_grad_noalloc(pet_geom g, int subset, const float *x, const void *y, int y_dtype,
                                              const float *add, const float *mult, float *grad_out, double *kl_out,
                                              void *stream) {
    if (!g || !x || !y || !grad_out) return fail(PET_E_ARG, "pet_subset_grad_noalloc: null argument");
    if (subset < -1 || subset >= g->d.n_subsets) return fail(PET_E_ARG, "pet_subset_grad_noalloc: subset out of range");
    if (y_dtype != PET_Y_F32 && y_dtype != PET_Y_U16 && y_dtype != PET_Y_U8)
        return fail(PET_E_ARG, "pet_subset_grad_noalloc: bad y dtype");
    const Layout L = layout_of(g, subset);
    if (L.total > SCRATCH_BYTES)
        return fail(PET_E_ARG, "pet_subset_grad_noalloc: this geometry needs " + std::to_string(L.total) +
                                   " bytes of work buffers, more than the static scratch of " +
                                   std::to_string(SCRATCH_BYTES) + " bytes");
    void *base = nullptr;
    pet_status st = noalloc_scratch(g->device, &base);
    if (st != PET_OK) return st;
    unsigned char *b = static_cast<unsigned char *>(base);
    SheetBufs w{reinterpret_cast<float *>(b + L.t0), reinterpret_cast<float *>(b + L.t1),
                reinterpret_cast<float *>(b + L.g0), reinterpret_cast<float *>(b + L.g1),
                g->psf_passes ? reinterpret_cast<float *>(b + L.psf_a) : nullptr,
                g->psf_passes ? reinterpret_cast<float *>(b + L.psf_b) : nullptr};
    double *partial = reinterpret_cast<double *>(b + L.partial);
    hipStream_t s = (hipStream_t)stream;
    if (checking(g)) {
        st = check_data(g, reinterpret_cast<unsigned *>(b + L.counts), s, "pet_subset_grad_noalloc", x, y, y_dtype,
                        add, mult);
        if (st != PET_OK) return st;
    }

    // the array keeps the previous call's contents (possibly another layout):
    // the image sheets' zero borders and the gradient sheets are cleared here
    hipError_t e = launch_clear_image_sheets(g, w, s);
    if (e == hipSuccess) e = launch_to_sheets_b(g, w, x, s);
    if (e == hipSuccess) e = launch_zero_sheets_b(g, w, s);
    ProjArgs a = subset_proj_args(g, subset);
    a.T0 = w.T0;
    a.T1 = w.T1;
    a.G0 = w.G0;
    a.G1 = w.G1;
    a.y = y;
    a.y_dtype = y_dtype;
    a.add = add;
    a.mult = mult;
    a.partial = kl_out ? partial : nullptr;
    if (e == hipSuccess) e = launch_line_kernel(g, M_GRAD, subset, a, s);
    if (e == hipSuccess && kl_out) e = launch_reduce_sum(partial, n_line_blocks(g, subset), kl_out, 0, s);
    if (e == hipSuccess) e = launch_from_sheets_b(g, w, grad_out, 0, s);
    return hip_check(e, "pet_subset_grad_noalloc");
}
