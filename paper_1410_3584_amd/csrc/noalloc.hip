// nlf_potential_noalloc: the potential evaluation of nlf_potential with its per-call scratch (the
// oversampled grids, the node values, the 3D node accumulators, the moments and their partial
// sums) taken from a fixed device array of the library instead of the plan's workspace, for
// callers that cannot allocate device memory.  The call itself allocates nothing: no hipMalloc, no
// hipFree, no allocating library routine.
//
// The array is a file-scope __device__ object.  Every GPU the library runs on holds its own copy,
// at its own address, from the loading of the code object until the process ends.  In host code its
// name is only a host-side handle, so the device address is fetched once per device with
// hipGetSymbolAddress (first call on that device, that device current) and kept; kernels and
// copies only ever receive that address.
#include <mutex>

#include "nlf_internal.h"

namespace nlf {

static __device__ __align__(256) unsigned char scratch[NLF_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device
static int scratch_address(void** out) {
    int dev = -1;
    NLF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(NLF_EUNSUPPORTED, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return set_error(NLF_EHIP, "hipGetSymbolAddress of the no-allocation scratch failed on device %d: %s", dev,
                             hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return NLF_OK;
}

// consecutive 256-byte aligned pieces of the scratch array
struct Carve {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t at = (off + 255) & ~(size_t)255;
        off = at + bytes;
        return at;
    }
};

// the buffers a potential evaluation writes before it reads them, in the plan and in the scratch
struct ScratchLayout {
    size_t grid_a, grid_b, cbuf, iacc, mom, red, total;
};

static ScratchLayout layout_of(const nlf_plan* p) {
    Carve c;
    ScratchLayout s{};
    s.grid_a = c.take((size_t)p->batch * p->G * elem_size(p->prec));
    s.grid_b = c.take((size_t)p->batch * p->G * elem_size(p->t1_prec));
    s.cbuf = c.take((size_t)p->batch * p->Mh * elem_size(p->prec));
    s.iacc = p->iacc ? c.take((size_t)p->batch * p->Mh * 2 * sizeof(double)) : 0;
    s.mom = c.take((size_t)p->batch * 4 * sizeof(double));
    s.red = c.take(p->red_bytes);
    s.total = c.off;
    return s;
}

// Points the plan's per-call buffers at the scratch for the lifetime of the object.
struct ScratchSwap {
    nlf_plan* p;
    void *ga, *gb, *cb;
    double *ia, *mo, *rd;
    ScratchSwap(nlf_plan* pl, unsigned char* base, const ScratchLayout& s)
        : p(pl), ga(pl->grid_a), gb(pl->grid_b), cb(pl->cbuf), ia(pl->iacc), mo(pl->mom), rd(pl->red) {
        p->grid_a = base + s.grid_a;
        p->grid_b = base + s.grid_b;
        p->cbuf = base + s.cbuf;
        if (p->iacc) p->iacc = reinterpret_cast<double*>(base + s.iacc);
        p->mom = reinterpret_cast<double*>(base + s.mom);
        p->red = reinterpret_cast<double*>(base + s.red);
    }
    ~ScratchSwap() {
        p->grid_a = ga;
        p->grid_b = gb;
        p->cbuf = cb;
        p->iacc = ia;
        p->mom = mo;
        p->red = rd;
    }
};

}  // namespace nlf

using namespace nlf;

extern "C" int nlf_potential_noalloc(nlf_plan* p, const void* rho, void* u) {
    clear_error();
    if (!p || !rho || !u) return set_error(NLF_EINVAL, "plan, rho and u must not be NULL");
    if (rho == u) return set_error(NLF_EINVAL, "rho and u may not alias");
    // a split's ball keeps its spectrum zero outside its band from plan creation on, and a
    // deterministic plan its per-item partial sums: neither fits a scratch that other calls reuse
    if (p->sub) return set_error(NLF_EUNSUPPORTED, "nlf_potential_noalloc does not take split plans");
    if (p->deterministic) return set_error(NLF_EUNSUPPORTED, "nlf_potential_noalloc does not take deterministic plans");
    const ScratchLayout s = layout_of(p);
    if (s.total > (size_t)NLF_NOALLOC_MAX_BYTES)
        return set_error(NLF_EINVAL, "this plan needs %zu bytes of scratch per call; nlf_potential_noalloc holds at most "
                         "%llu (NLF_NOALLOC_MAX_BYTES)", s.total, (unsigned long long)NLF_NOALLOC_MAX_BYTES);
    void* base = nullptr;
    NLF_TRY(scratch_address(&base));
    // every scratch buffer is written before it is read within the call (grid_b and the 3D node
    // accumulators are cleared by kernels of the call itself), so the previous call's contents
    // never leak into this one
    ScratchSwap swap(p, static_cast<unsigned char*>(base), s);
    if (p->check_finite) {
        int seen = 0;
        NLF_TRY(read_nonfinite(p, &seen));
    }
    NLF_TRY(potential(p, rho, u));
    if (p->check_finite) {
        int seen = 0;
        NLF_TRY(read_nonfinite(p, &seen));
        if (seen) return set_error(NLF_ENONFINITE, "the density holds a NaN or Inf value");
    }
    return NLF_OK;
}
