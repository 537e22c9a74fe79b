// Plan construction: Fourier-space quadrature nodes (Sec. 2.1, Eq. 'ifft'), Gaussian-gridding
// parameters of the NUFFT, node binning on the oversampled grid, workspace allocation.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "exec.h"
#include "nlf_internal.h"

namespace nlf {

static thread_local char g_err[512] = "";

int set_error(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}
void clear_error() { g_err[0] = 0; }

size_t elem_size(int prec) { return prec == NLF_F64 ? 16 : 8; }

XcdSplit xcd_split(const std::vector<long long>& cost) {
    XcdSplit xs{};
    const int n = (int)cost.size();
    long long total = 0;
    for (long long c : cost) total += c;
    long long acc = 0;
    int x = 1;
    for (int i = 0; i < n && x < 8; ++i) {
        acc += cost[i];
        while (x < 8 && acc * 8 >= total * x) xs.s[x++] = i + 1;
    }
    while (x <= 8) xs.s[x++] = n;
    xs.per = 1;
    for (int k = 0; k < 8; ++k) xs.per = std::max(xs.per, xs.s[k + 1] - xs.s[k]);
    return xs;
}

// Estimated cost of a gather work item or an interpolation chunk: its nodes plus a fixed part (the
// tile's write-back, the window's staging).
constexpr long long kItemFixed = 64;
constexpr long long kChunkFixed = 64;
// Within each XCD's range the entries with the most nodes go first, so that the range does not end
// on a long one (512^2 FP64: interpolation 42.8 -> 39.6 us, spreading 57.3 -> 55.7 us).
template <class E>
static void heavy_first(std::vector<E>& v, const XcdSplit& xs) {
    for (int x = 0; x < 8; ++x)
        std::stable_sort(v.begin() + xs.s[x], v.begin() + xs.s[x + 1],
                         [](const E& a, const E& b) { return a.count > b.count; });
}

// Work items of the gather kernels: the candidates of each tile cut into pieces of <= cap.
int set_items(nlf_plan* p, int cap, bool bins) {
    std::vector<GItem> items;
    const long long ntiles = (long long)p->gng[0] * p->gng[1] * p->gng[2];
    const std::vector<long long>& off = bins ? p->vtile_off : p->gtile_off;
    for (long long t = 0; t < ntiles; ++t) {
        const long long beg = off[t], end = off[t + 1];
        const int g2 = (int)(t % p->gng[2]);
        const int g1 = (int)((t / p->gng[2]) % p->gng[1]);
        const int g0 = (int)(t / ((long long)p->gng[2] * p->gng[1]));
        for (long long s0 = beg; s0 < end; s0 += cap) {
            GItem it;
            it.g0 = g0;
            it.g1 = g1;
            it.g2 = g2;
            it.count = (int)std::min<long long>(cap, end - s0);
            it.start = bins ? s0 - beg : s0;   // bins: offset within the tile's candidate stream
            it.only = (end - beg <= cap) ? 1 : 0;
            it.slot = -1;
            items.push_back(it);
        }
    }
    if ((long long)items.size() > p->gitems_cap)
        return set_error(NLF_EINVAL, "work-item size %d below the allocated minimum", cap);
    // deterministic plans: the items of a tile of several store partial sums in consecutive
    // slots (assigned in tile order, before the items are reordered for the launch)
    std::vector<TileRed> tr;
    long long nslots = 0;
    if (p->deterministic) {
        for (size_t i = 0; i < items.size();) {
            size_t j = i;
            while (j < items.size() && items[j].g0 == items[i].g0 && items[j].g1 == items[i].g1 &&
                   items[j].g2 == items[i].g2)
                ++j;
            if (!items[i].only) {
                tr.push_back({items[i].g0, items[i].g1, items[i].g2, (int)nslots, (int)(j - i)});
                for (size_t k = i; k < j; ++k) items[k].slot = (int)nslots++;
            }
            i = j;
        }
    }
    XcdSplit xs;
    {
        std::vector<long long> cost(items.size());
        for (size_t i = 0; i < items.size(); ++i) cost[i] = items[i].count + kItemFixed;
        xs = xcd_split(cost);
        heavy_first(items, xs);
    }
    NLF_HIP(hipStreamSynchronize(p->stream));   // no kernel of the plan may still read the items
    if (!items.empty()) {
        NLF_HIP(hipMemcpyAsync(p->gitems, items.data(), items.size() * sizeof(GItem), hipMemcpyHostToDevice,
                               p->stream));
        NLF_HIP(hipStreamSynchronize(p->stream));   // `items` is released on return
    }
    if (p->deterministic) {
        if (nslots > p->pscratch_slots) {
            NLF_TRY(dev_alloc(p, (void**)&p->pscratch, (size_t)p->batch * nslots * 256 * sizeof(double)));
            p->pscratch_slots = nslots;
        }
        if ((long long)tr.size() > p->tred_cap) {
            NLF_TRY(dev_alloc(p, (void**)&p->tred, tr.size() * sizeof(TileRed)));
            p->tred_cap = (long long)tr.size();
        }
        if (!tr.empty()) {
            NLF_HIP(hipMemcpyAsync(p->tred, tr.data(), tr.size() * sizeof(TileRed), hipMemcpyHostToDevice, p->stream));
            NLF_HIP(hipStreamSynchronize(p->stream));
        }
        p->nslots = nslots;
        p->ntred = (int)tr.size();
    }
    p->ngitems = (int)items.size();
    p->item_split = xs;
    p->item_cap = cap;
    p->items_bins = bins ? 1 : 0;
    return NLF_OK;
}

Recorder*& recorder() {
    thread_local Recorder* r = nullptr;
    return r;
}

// NLF_MAX_WORKSPACE_BYTES: an optional cap on a plan's own device memory (0 or unset: none)
static long long workspace_cap() {
    const char* v = std::getenv("NLF_MAX_WORKSPACE_BYTES");
    if (!v || !*v) return 0;
    char* end = nullptr;
    const long long c = std::strtoll(v, &end, 10);
    return (end && *end == '\0' && c > 0) ? c : 0;
}

int dev_alloc(nlf_plan* p, void** ptr, size_t bytes) {
    *ptr = nullptr;
    if (bytes == 0) bytes = 256;
    const long long cap = workspace_cap();
    if (cap > 0 && p->workspace_bytes + (long long)bytes > cap)
        return set_error(NLF_ENOMEM, "allocating %zu bytes would take the plan's workspace to %lld bytes, above "
                         "NLF_MAX_WORKSPACE_BYTES = %lld", bytes, p->workspace_bytes + (long long)bytes, cap);
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *ptr = nullptr;
        return set_error(NLF_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    p->owned.push_back(*ptr);
    p->workspace_bytes += (long long)bytes;
    return NLF_OK;
}

// n-point Gauss-Legendre rule on [-1,1] by Newton's iteration on the three-term recurrence of
// the Legendre polynomials, in long double; nodes ascending, mirrored so that t[n-1-i] = -t[i]
// exactly (the node set must be symmetric for the k -> -k pairing of the quadrature nodes).
static void gauss_legendre(int n, std::vector<double>& t, std::vector<double>& w) {
    t.assign(n, 0.0);
    w.assign(n, 0.0);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        long double x = cosl(pi * (i + 0.75L) / (n + 0.5L));
        long double dp = 0;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1, p1 = x;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = x; p0 = 1; }
            dp = n * (x * p1 - p0) / (x * x - 1);
            long double dx = p1 / dp;
            x -= dx;
            if (fabsl(dx) < 1e-19L) break;
        }
        // recompute the derivative at the converged node for the weight
        long double p0 = 1, p1 = x;
        for (int k = 2; k <= n; ++k) {
            long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) { p1 = x; p0 = 1; }
        dp = n * (x * p1 - p0) / (x * x - 1);
        long double wi = 2.0L / ((1 - x * x) * dp * dp);
        // x is the i-th largest node
        t[n - 1 - i] = (double)x;
        t[i] = -(double)x;
        w[n - 1 - i] = (double)wi;
        w[i] = (double)wi;
    }
    if (n % 2 == 1) t[n / 2] = 0.0;
}

static bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// E1(z) + ln z for z >= 0 in long double: the power series -gamma - sum_{k>=1} (-z)^k / (k k!)
// (Abramowitz & Stegun 5.1.11) below z = 1, the continued fraction of E1 (A&S 5.1.22, modified Lentz
// evaluation) above; E1 is dropped beyond z = 45 where it is below the rounding of ln z.
static long double e1_plus_log(long double z) {
    const long double egamma = 0.577215664901532860606512090082402431L;
    if (z < 1.0L) {
        long double term = 1.0L, sum = 0.0L;
        for (int k = 1; k < 60; ++k) {
            term *= -z / k;
            long double t = term / k;
            sum += t;
            if (fabsl(t) <= 1e-21L * fabsl(sum)) break;
        }
        return -egamma - sum;
    }
    if (z > 45.0L) return logl(z);
    const long double tiny = 1e-4000L;
    long double b = z + 1.0L, c = 1.0L / tiny, d = 1.0L / b, h = d;
    for (int i = 1; i < 1000; ++i) {
        long double an = -(long double)i * i;
        b += 2.0L;
        d = 1.0L / (an * d + b);
        c = b + an / c;
        long double del = c * d;
        h *= del;
        if (fabsl(del - 1.0L) < 1e-19L) break;
    }
    return h * expl(-z) + logl(z);
}

// Every initialisation of device memory goes through the plan's stream: the stream may be a
// non-blocking one, which the legacy default stream (where hipMemcpy and hipMemset run) does not
// order against, so a plain copy or fill could land after the plan's first kernels.
static int upload(nlf_plan* p, void** dst, const void* src, size_t bytes) {
    NLF_TRY(dev_alloc(p, dst, bytes));
    NLF_HIP(hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, p->stream));
    NLF_HIP(hipStreamSynchronize(p->stream));   // the host table may be released on return
    return NLF_OK;
}

template <typename T>
static int upload_twiddles(nlf_plan* p, void** dst, int n) {
    std::vector<T> tw(2 * (size_t)n);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int t = 0; t < n; ++t) {
        long double a = -2.0L * pi * t / n;
        tw[2 * t] = (T)cosl(a);
        tw[2 * t + 1] = (T)sinl(a);
    }
    return upload(p, dst, tw.data(), tw.size() * sizeof(T));
}

// erfcx(a) = e^{a^2} erfc(a) for a >= 0, the closed form of the confined kernel's symbol x Jacobian
//   (2/pi) int_0^inf e^{-a^2 s^2} / (1 + s^2) ds  (Eq. '2Dw1' with a = eps |k| / sqrt 2).
// a < 8: e^{a^2} erfc(a) with a^2 split exactly into hi + lo (fma), e^{a^2} = e^{hi} (1 + lo).
// a >= 8: Laplace's continued fraction for the complementary error function (Abramowitz and
// Stegun 7.1.14), sqrt(pi) erfcx(a) = 1/(a + (1/2)/(a + 1/(a + (3/2)/(a + 2/(a + ...))))), summed
// from the 60th level up (at a >= 8 it has converged to rounding long before).
static double erfcx_host(double a) {
    if (a < 8.0) {
        const double hi = a * a, lo = std::fma(a, a, -hi);
        return std::exp(hi) * (1.0 + lo) * std::erfc(a);
    }
    double f = a;
    for (int j = 60; j >= 1; --j) f = a + 0.5 * j / f;
    return 1.0 / (std::sqrt(3.14159265358979323846) * f);
}

static int plan_create(const nlf_box* box, int kernel, const nlf_opts* opts, void* stream, double pweight_a,
                       nlf_plan** out);
static int build(nlf_plan* p, const nlf_box* box, int kernel, const nlf_opts* o);

// Split evaluation (Sec. 2.1, Eq. '3.9'), 3D Coulomb.  This plan keeps only what I1 needs: the
// oversampled grid, its twiddles and unit pre/post-correction tables (so that the type-2 and
// type-1 FFT passes become the plain zero-padded forward FFT and the truncating inverse FFT of a
// cyclic convolution).  I2 is a ball plan (`sub`) of radius P2 whose node weights carry p(k).
static int build_split(nlf_plan* p, const nlf_box* box, int kernel, const nlf_opts* o) {
    if (kernel != NLF_COULOMB3D) return set_error(NLF_EUNSUPPORTED, "the split evaluation is for NLF_COULOMB3D");
    if (o->P > 0 || o->sigma > 0) return set_error(NLF_EINVAL, "a split plan takes no P or sigma");
    double Lmin = p->L[0], D2 = 0;
    for (int i = 0; i < 3; ++i) {
        Lmin = std::min(Lmin, p->L[i]);
        D2 += 4.0 * p->L[i] * p->L[i];
    }
    p->split = 1;
    p->split_a = (o->split_a > 0) ? o->split_a : (5.5 / Lmin) * (5.5 / Lmin);
    p->split_P2 = std::sqrt(34.5 * p->split_a);
    if (p->split_P2 > p->P * (1 + 1e-12))
        return set_error(NLF_EUNSUPPORTED, "grid too coarse for the split: pi/max(h) = %g < P2 = sqrt(34.5 a) = %g",
                         p->P, p->split_P2);
    // ball rule: 0.75 of the largest phase P2 D / 2 across the box, plus 8 (converged to rounding
    // from about 0.65 on densities in opposite corners of the box)
    const int nr = (int)std::ceil(0.375 * p->split_P2 * std::sqrt(D2)) + 8;
    nlf_opts so = *o;
    so.split = 0;
    so.split_a = 0;
    so.P = p->split_P2;
    so.n_r = o->n_r > 0 ? o->n_r : nr;
    so.n_theta = o->n_theta > 0 ? o->n_theta : nr;
    so.n_phi = o->n_phi > 0 ? o->n_phi : 2 * nr;
    NLF_TRY(plan_create(box, kernel, &so, p->stream, p->split_a, &p->sub));
    // the ball's spectrum band: node positions reach 2 L_i P2 / pi oversampled cells from the
    // origin, stencils msp more and whole gather tiles (<= 8 cells) one more; rounded up to whole
    // 16-column blocks.  Cells outside it are never read or written by the ball's FFT passes.
    {
        nlf_plan* b = p->sub;
        double reach = 0;
        for (int i = 0; i < 3; ++i) reach = std::max(reach, 2.0 * p->L[i] * p->split_P2 / 3.14159265358979323846);
        int band = ((int)std::ceil(reach) + b->msp + 9 + 15) / 16 * 16;
        bool fits = true;
        for (int i = 0; i < 3; ++i) fits = fits && 2 * band <= b->Mr[i] / 2;
        if (fits) {
            b->band = band;
            NLF_HIP(hipMemsetAsync(b->grid_a, 0, (size_t)b->batch * b->G * elem_size(b->prec), b->stream));
        }
    }
    p->n_r = p->sub->n_r;
    p->n_theta = p->sub->n_theta;
    p->n_phi = p->sub->n_phi;
    p->M = p->sub->M;
    p->Mh = p->sub->Mh;

    const size_t es = elem_size(p->prec);
    p->t1_prec = p->prec;
    NLF_TRY(dev_alloc(p, &p->grid_a, (size_t)p->batch * p->G * es));
    p->grid_b = p->grid_a;   // the inverse transform runs in place on the multiplied spectrum
    for (int i = 0; i < p->dim; ++i) {
        std::vector<double> one(p->n[i], 1.0);
        NLF_TRY(upload(p, (void**)&p->dec[i], one.data(), one.size() * sizeof(double)));
        if (p->prec == NLF_F64) {
            NLF_TRY(upload_twiddles<double>(p, &p->tw_big[i], p->Mr[i]));
            NLF_TRY(upload_twiddles<double>(p, &p->tw_small[i], p->n[i]));
        } else {
            NLF_TRY(upload_twiddles<float>(p, &p->tw_big[i], p->Mr[i]));
            NLF_TRY(upload_twiddles<float>(p, &p->tw_small[i], p->n[i]));
        }
        p->tw_t1[i] = p->tw_big[i];
    }
    {   // the multiply's axis-0 factor exp(-k0^2 / a), k0 the centred frequency of row r
        std::vector<double> e0(p->Mr[0]);
        const double dk0 = 2.0 * 3.14159265358979323846 / (p->Mr[0] * p->h[0]);
        for (int r = 0; r < p->Mr[0]; ++r) {
            const double k0 = (r < p->Mr[0] / 2 ? r : r - p->Mr[0]) * dk0;
            e0[r] = std::exp(-k0 * k0 / p->split_a);
        }
        NLF_TRY(upload(p, (void**)&p->conv_e0, e0.data(), e0.size() * sizeof(double)));
    }
    NLF_TRY(dev_alloc(p, (void**)&p->mom, (size_t)p->batch * 4 * sizeof(double)));
    p->red_bytes = (size_t)p->batch * 1024 * 8 * sizeof(double);
    NLF_TRY(dev_alloc(p, (void**)&p->red, p->red_bytes));
    NLF_TRY(dev_alloc(p, (void**)&p->nf_flag, sizeof(int)));
    NLF_HIP(hipMemsetAsync(p->nf_flag, 0, sizeof(int), p->stream));
    p->sub->nf_flag = p->nf_flag;   // both density loads of a split (I1's and the ball's) report here
    p->spread_mode = p->sub->spread_mode;
    return NLF_OK;
}

static int build(nlf_plan* p, const nlf_box* box, int kernel, const nlf_opts* o) {
    const double pi = 3.14159265358979323846;
    p->dim = box->dim;
    p->kernel = kernel;
    if (p->dim != 2 && p->dim != 3) return set_error(NLF_EUNSUPPORTED, "dim must be 2 or 3 (got %d)", p->dim);
    if ((kernel == NLF_COULOMB3D && p->dim != 3) ||
        ((kernel == NLF_COULOMB2D || kernel == NLF_LAPLACE2D || kernel == NLF_CONFINED2D) && p->dim != 2))
        return set_error(NLF_EUNSUPPORTED, "kernel %d does not match dim %d", kernel, p->dim);
    if (kernel < NLF_COULOMB3D || kernel > NLF_CONFINED2D)
        return set_error(NLF_EINVAL, "unknown kernel %d", kernel);
    if (kernel == NLF_CONFINED2D) {
        p->eps = o ? o->eps : 0.0;
        if (!(p->eps > 0) || !std::isfinite(p->eps))
            return set_error(NLF_EINVAL, "the confined Coulomb kernel needs opts.eps > 0 (got %g)", p->eps);
    }
    p->prec = o ? o->prec : NLF_F64;
    if (p->prec != NLF_F64 && p->prec != NLF_F32) return set_error(NLF_EINVAL, "prec must be NLF_F64 or NLF_F32");
    p->deterministic = (o && o->deterministic) ? 1 : 0;
    p->check_finite = (o && o->check_finite) ? 1 : 0;
    p->batch = (o && o->batch > 0) ? o->batch : 1;
    p->N = 1;
    p->G = 1;
    double hmax = 0;
    for (int i = 0; i < 3; ++i) {
        if (i >= p->dim) { p->n[i] = 1; p->Mr[i] = 1; p->L[i] = 0; p->h[i] = 0; continue; }
        int ni = box->n[i];
        if (!pow2(ni) || ni < 8 || ni > 1024)
            return set_error(NLF_EUNSUPPORTED, "n[%d] = %d must be a power of two in [8, 1024]", i, ni);
        if (!(box->L[i] > 0)) return set_error(NLF_EINVAL, "L[%d] must be positive", i);
        p->n[i] = ni;
        p->Mr[i] = 2 * ni;
        p->L[i] = box->L[i];
        p->h[i] = 2.0 * box->L[i] / ni;
        hmax = std::max(hmax, p->h[i]);
        p->N *= ni;
        p->G *= 2 * ni;
    }
    p->P = (o && o->P > 0) ? o->P : pi / hmax;
    if (p->P > pi / hmax * (1 + 1e-12))
        return set_error(NLF_EINVAL, "P = %g exceeds the grid's Nyquist radius pi/max(h) = %g", p->P, pi / hmax);
    p->n_r = (o && o->n_r > 0) ? o->n_r : p->n[0];
    p->n_theta = (p->dim == 3) ? ((o && o->n_theta > 0) ? o->n_theta : p->n[0]) : 1;
    p->n_phi = (o && o->n_phi > 0) ? o->n_phi : 2 * p->n[0];
    if (p->n_phi % 2) return set_error(NLF_EINVAL, "n_phi must be even (k -> -k pairing)");
    p->sigma = (o && o->sigma > 0) ? o->sigma : 6.0 * std::sqrt(2.0) / p->P;
    p->msp = (o && o->msp > 0) ? o->msp : (p->prec == NLF_F64 ? 12 : 7);
    if (p->msp < 2 || p->msp > kMaxMsp) return set_error(NLF_EINVAL, "msp must be in [2, %d]", kMaxMsp);
    p->M = (long long)p->n_r * p->n_theta * p->n_phi;
    p->Mh = p->M / 2;

    // Gaussian gridding with oversampling 2: tau_i = pi msp / (n_i^2 R (R - 1/2)), R = 2.  In units
    // of oversampled cells the spreading Gaussian is exp(-alpha (p - delta)^2), alpha = 3 pi / (4 msp),
    // independent of n_i.
    p->gc.alpha = 3.0 * pi / (4.0 * p->msp);
    for (int q = 0; q < 2 * kMaxMsp; ++q) {
        int pp = q - p->msp + 1;
        p->gc.e3[q] = (q < 2 * p->msp) ? std::exp(-p->gc.alpha * pp * pp) : 0.0;
    }
    p->st2 = 1.0;
    p->post = 1.0;
    for (int i = 0; i < p->dim; ++i) {
        p->st2 *= p->h[i] / p->Mr[i];
        p->post /= p->Mr[i];
    }

    // tiles: node bins of the gather-tile shape, 8 x 16 cells (2D) or 8 x 4 x 4 (3D): the 2D
    // interpolation stages one bin's window per workgroup, and the neighbour-bin gather reads a
    // tile's candidates as whole bins
    for (int i = 0; i < 3; ++i) {
        int t = (p->dim == 2) ? (i == 0 ? 8 : 16) : (i == 0 ? 8 : 4);
        if (i >= p->dim) t = 1;
        p->tile[i] = std::min(t, p->Mr[i]);
        p->window[i] = (i < p->dim) ? p->tile[i] + 2 * p->msp - 1 : 1;
    }
    if (o && o->split) return build_split(p, box, kernel, o);

    // ---- quadrature nodes (canonical order) -----------------------------------------------
    std::vector<double> tr, wr, mu, wmu;
    gauss_legendre(p->n_r, tr, wr);
    for (int a = 0; a < p->n_r; ++a) {
        tr[a] = 0.5 * p->P * (tr[a] + 1.0);
        wr[a] = 0.5 * p->P * wr[a];
    }
    if (p->dim == 3) gauss_legendre(p->n_theta, mu, wmu);
    else { mu.assign(1, 0.0); wmu.assign(1, 1.0); }
    std::vector<double> cph(p->n_phi), sph(p->n_phi);
    const long double lpi = 3.141592653589793238462643383279502884L;
    for (int c = 0; c < p->n_phi; ++c) {
        long double a = 2.0L * lpi * c / p->n_phi;
        cph[c] = (double)cosl(a);
        sph[c] = (double)sinl(a);
    }
    const double wphi = 2.0 * pi / p->n_phi;
    p->k_host.assign((size_t)p->M * p->dim, 0.0);
    p->w_host.assign((size_t)p->M, 0.0);
    for (int a = 0; a < p->n_r; ++a)
        for (int b = 0; b < p->n_theta; ++b)
            for (int c = 0; c < p->n_phi; ++c) {
                size_t m = ((size_t)a * p->n_theta + b) * p->n_phi + c;
                double r = tr[a];
                if (p->dim == 2) {
                    p->k_host[2 * m] = r * cph[c];
                    p->k_host[2 * m + 1] = r * sph[c];
                    p->w_host[m] = wr[a] * wphi;
                } else {
                    double st = std::sqrt((1.0 - mu[b]) * (1.0 + mu[b]));
                    p->k_host[3 * m] = r * st * cph[c];
                    p->k_host[3 * m + 1] = r * st * sph[c];
                    p->k_host[3 * m + 2] = r * mu[b];
                    p->w_host[m] = wr[a] * wmu[b] * wphi;
                }
            }

    // ---- half node set, binning ----------------------------------------------------------------
    const int hphi = p->n_phi / 2;
    const long long Mh = p->Mh;
    std::vector<double> sh[3];
    for (int i = 0; i < p->dim; ++i) sh[i].resize(Mh);
    std::vector<int> bin(Mh);
    int nb[3];
    for (int i = 0; i < 3; ++i) nb[i] = (i < p->dim) ? p->Mr[i] / p->tile[i] : 1;
    const long long nbins = (long long)nb[0] * nb[1] * nb[2];
    std::vector<int> cnt(nbins + 1, 0);
    for (long long hm = 0; hm < Mh; ++hm) {
        long long ab = hm / hphi;
        int c = (int)(hm % hphi);
        size_t m = (size_t)ab * p->n_phi + c;
        int bt[3] = {0, 0, 0};
        for (int i = 0; i < p->dim; ++i) {
            double s = 2.0 * p->L[i] * p->k_host[(size_t)p->dim * m + i] / pi;
            sh[i][hm] = s;
            long long l0 = (long long)std::floor(s);
            long long lm = ((l0 % p->Mr[i]) + p->Mr[i]) % p->Mr[i];
            bt[i] = (int)(lm / p->tile[i]);
        }
        int bid = (bt[0] * nb[1] + bt[1]) * nb[2] + bt[2];
        bin[hm] = bid;
        cnt[bid + 1]++;
    }
    for (long long b = 0; b < nbins; ++b) cnt[b + 1] += cnt[b];
    std::vector<int> order(Mh);
    {
        std::vector<int> pos(cnt.begin(), cnt.end() - 1);
        for (long long hm = 0; hm < Mh; ++hm) order[pos[bin[hm]]++] = (int)hm;
    }
    if (p->dim == 2) {
        // within a 2D bin, order the nodes by their axis-1 cell (then axis-0 cell): 16 consecutive
        // nodes then span few columns, and the interpolation multiplies only the columns they touch
        auto cell = [&](int hm, int i) {
            long long l0 = (long long)std::floor(sh[i][hm]);
            return (int)(((l0 % p->Mr[i]) + p->Mr[i]) % p->Mr[i]);
        };
        for (long long b = 0; b < nbins; ++b)
            std::stable_sort(order.begin() + cnt[b], order.begin() + cnt[b + 1], [&](int a, int c) {
                const int ya = cell(a, 1), yc = cell(c, 1);
                return ya != yc ? ya < yc : cell(a, 0) < cell(c, 0);
            });
    }
    std::vector<Chunk> chunks;
    for (long long b = 0; b < nbins; ++b) {
        int beg = cnt[b], end = cnt[b + 1];
        int bt2 = (int)(b % nb[2]);
        int bt1 = (int)((b / nb[2]) % nb[1]);
        int bt0 = (int)(b / ((long long)nb[2] * nb[1]));
        for (int s = beg; s < end; s += kChunk) {
            Chunk ch;
            ch.start = s;
            ch.count = std::min(kChunk, end - s);
            ch.t0 = bt0;
            ch.t1 = bt1;
            ch.t2 = bt2;
            ch.pad = 0;
            chunks.push_back(ch);
        }
    }
    p->nchunks = (int)chunks.size();
    {
        std::vector<long long> cost(chunks.size());
        for (size_t i = 0; i < chunks.size(); ++i) cost[i] = chunks[i].count + kChunkFixed;
        p->chunk_split = xcd_split(cost);
        heavy_first(chunks, p->chunk_split);
    }

    // ---- candidate lists for the output-driven spreading ------------------------------------
    // A node at l0 touches cells (l0 + p) mod Mr, p = -msp+1..msp, along each axis; list it under
    // every gather tile its stencil overlaps.  Plans whose list would exceed kMaxCand entries keep
    // the scatter kernels.
    {
        const long long kMaxCand = 400000000LL;
        int gt[3], ng[3];
        for (int i = 0; i < 3; ++i) {
            gt[i] = (i >= p->dim) ? 1 : (i == 0 ? 8 : (p->dim == 2 ? 16 : 4));   // Mr >= 16 always
            p->gtile[i] = gt[i];
            ng[i] = (i < p->dim) ? p->Mr[i] / gt[i] : 1;
        }
        const long long ntiles = (long long)ng[0] * ng[1] * ng[2];
        auto axis_tiles = [&](double s, int i, int* out) -> int {
            long long l0 = (long long)std::floor(s);
            int cnt = 0;
            // a stencil longer than Mr - gt + 1 can start and end in one tile while wrapping
            // through the others: list every tile of the axis
            if (2 * p->msp + gt[i] > p->Mr[i]) {
                for (int t = 0; t < ng[i]; ++t) out[cnt++] = t;
                return cnt;
            }
            int first = (int)((((l0 - p->msp + 1) % p->Mr[i]) + p->Mr[i]) % p->Mr[i]) / gt[i];
            int last = (int)((((l0 + p->msp) % p->Mr[i]) + p->Mr[i]) % p->Mr[i]) / gt[i];
            int t = first;
            while (true) {
                out[cnt++] = t;
                if (t == last || cnt == ng[i]) break;
                t = (t + 1) % ng[i];
            }
            return cnt;
        };
        std::vector<long long> tcount(ntiles + 1, 0);
        long long total = 0;
        std::vector<int> tl[3];
        for (int i = 0; i < 3; ++i) tl[i].resize(std::max(ng[i], 1));
        for (long long j = 0; j < Mh && total <= kMaxCand; ++j) {
            int hm = order[j];
            int c3[3] = {1, 1, 1};
            for (int i = 0; i < p->dim; ++i) c3[i] = axis_tiles(sh[i][hm], i, tl[i].data());
            for (int a = 0; a < c3[0]; ++a)
                for (int b = 0; b < c3[1]; ++b)
                    for (int c = 0; c < c3[2]; ++c) {
                        int t0 = p->dim > 0 ? tl[0][a] : 0, t1 = tl[1][b], t2 = p->dim == 3 ? tl[2][c] : 0;
                        long long tid = ((long long)t0 * ng[1] + t1) * ng[2] + t2;
                        tcount[tid + 1]++;
                    }
            total += (long long)c3[0] * c3[1] * c3[2];
        }
        if (total <= kMaxCand) {
            for (long long t = 0; t < ntiles; ++t) tcount[t + 1] += tcount[t];
            std::vector<int> cand(total);
            std::vector<long long> pos(tcount.begin(), tcount.end() - 1);
            for (long long j = 0; j < Mh; ++j) {
                int hm = order[j];
                int c3[3] = {1, 1, 1};
                for (int i = 0; i < p->dim; ++i) c3[i] = axis_tiles(sh[i][hm], i, tl[i].data());
                for (int a = 0; a < c3[0]; ++a)
                    for (int b = 0; b < c3[1]; ++b)
                        for (int c = 0; c < c3[2]; ++c) {
                            int t0 = tl[0][a], t1 = tl[1][b], t2 = p->dim == 3 ? tl[2][c] : 0;
                            long long tid = ((long long)t0 * ng[1] + t1) * ng[2] + t2;
                            cand[pos[tid]++] = (int)j;
                        }
            }
            p->gtile_off.assign(tcount.begin(), tcount.end());   // explicit lists
            p->use_gather = 1;
            NLF_TRY(upload(p, (void**)&p->gcand, cand.data(), std::max<size_t>(1, cand.size()) * sizeof(int)));
        }
        for (int i = 0; i < 3; ++i) p->gng[i] = ng[i];

        // Neighbour-bin gather: with node bins of the tile's shape, the nodes whose stencil can
        // reach tile t lie in the bins t + lo_i .. t + lo_i + nn_i - 1 per axis,
        // lo = floor(-msp / T), hi = floor((T + msp - 2) / T).  A tile's candidates are those bins'
        // node ranges, read in place (no per-pair list).  Needs more bins per axis than nn_i (no
        // bin counted twice) and Mr_i >= 2 msp + T_i (single-representative tile weights).
        bool impl = true;
        for (int i = 0; i < 3; ++i) {
            if (i >= p->dim) {
                p->impl_lo[i] = 0;
                p->impl_n[i] = 1;
                continue;
            }
            const int T = gt[i];
            const int lo = -((p->msp + T - 1) / T);        // floor(-msp / T)
            const int hi = (T + p->msp - 2) / T;
            p->impl_lo[i] = lo;
            p->impl_n[i] = hi - lo + 1;
            impl = impl && p->tile[i] == T && nb[i] >= p->impl_n[i] && p->Mr[i] >= 2 * p->msp + T;
        }
        if (impl && p->impl_n[0] * p->impl_n[1] * p->impl_n[2] <= kMaxNbrBins) {
            NLF_TRY(upload(p, (void**)&p->bin_off, cnt.data(), cnt.size() * sizeof(int)));
            p->vtile_off.assign(ntiles + 1, 0);
            for (long long t = 0; t < ntiles; ++t) {
                const int t2 = (int)(t % ng[2]), t1 = (int)((t / ng[2]) % ng[1]);
                const int t0 = (int)(t / ((long long)ng[2] * ng[1]));
                long long tot = 0;
                for (int a = 0; a < p->impl_n[0]; ++a) {
                    const int b0 = ((t0 + p->impl_lo[0] + a) % nb[0] + nb[0]) % nb[0];
                    for (int b = 0; b < p->impl_n[1]; ++b) {
                        const int b1 = ((t1 + p->impl_lo[1] + b) % nb[1] + nb[1]) % nb[1];
                        for (int c = 0; c < p->impl_n[2]; ++c) {
                            const int b2 = ((t2 + p->impl_lo[2] + c) % nb[2] + nb[2]) % nb[2];
                            const long long bid = ((long long)b0 * nb[1] + b1) * nb[2] + b2;
                            tot += cnt[bid + 1] - cnt[bid];
                        }
                    }
                }
                p->vtile_off[t + 1] = p->vtile_off[t] + tot;
            }
            p->gather_impl_ok = 1;
        }
        // one work-item buffer for every decomposition: room for the finest item sizes allowed
        // (256 candidates from the explicit lists, 512 from the neighbour bins)
        long long most = 1;
        if (p->use_gather) {
            long long m = 0;
            for (long long t = 0; t < ntiles; ++t) m += (p->gtile_off[t + 1] - p->gtile_off[t] + 255) / 256;
            most = std::max(most, m);
        }
        if (p->gather_impl_ok) {
            long long m = 0;
            for (long long t = 0; t < ntiles; ++t) m += (p->vtile_off[t + 1] - p->vtile_off[t] + 511) / 512;
            most = std::max(most, m);
        }
        if (p->use_gather || p->gather_impl_ok) {
            p->gitems_cap = most;
            NLF_TRY(dev_alloc(p, (void**)&p->gitems, (size_t)p->gitems_cap * sizeof(GItem)));
        }
        // default: the explicit lists with the largest items (1024 or 512 candidates) that still
        // leave 4096 work items per field, else 256-candidate items (the fastest on the 512^2
        // workloads measured: 1024 for FP64, msp 12, and 512 for FP32, msp 7; 256 on the small
        // solver grids; nlf_plan_autotune picks per plan); neighbour bins with 1024-candidate
        // items where the lists were not built
        if (p->deterministic && !p->use_gather && !p->gather_impl_ok)
            return set_error(NLF_EUNSUPPORTED, "a deterministic plan needs the gather spreading (lists or bins)");
        if (p->use_gather) {
            p->spread_mode = NLF_SPREAD_GATHER;
            int cap = 256;
            for (int c : {1024, 512}) {
                long long nit = 0;
                for (size_t t = 0; t + 1 < p->gtile_off.size(); ++t)
                    nit += (p->gtile_off[t + 1] - p->gtile_off[t] + c - 1) / c;
                if (nit >= 4096) {
                    cap = c;
                    break;
                }
            }
            NLF_TRY(set_items(p, cap, false));
        } else if (p->gather_impl_ok) {
            p->spread_mode = NLF_SPREAD_BINS;
            NLF_TRY(set_items(p, 1024, true));
        } else {
            p->spread_mode = NLF_SPREAD_SCATTER;
        }
    }

    // sorted per-node data
    std::vector<double> ss[3], wf(Mh), gk;
    for (int i = 0; i < p->dim; ++i) ss[i].resize(Mh);
    if (kernel == NLF_LAPLACE2D) gk.resize(Mh);
    const double inv2pid = std::pow(2.0 * pi, -p->dim);
    for (long long j = 0; j < Mh; ++j) {
        int hm = order[j];
        long long ab = hm / hphi;
        int c = hm % hphi;
        size_t m = (size_t)ab * p->n_phi + c;
        double kk = 0;
        for (int i = 0; i < p->dim; ++i) {
            ss[i][j] = sh[i][hm];
            double ki = p->k_host[(size_t)p->dim * m + i];
            kk += ki * ki;
        }
        double kmag = std::sqrt(kk);
        // u = Re sum_half 2 c_m e^{ikx}; c_m = (2pi)^-d w_m S_m (Eq. 'ifft' with the Jacobian
        // cancelled by the Coulomb symbol; Eq. 'phi2fourier' for the Laplace kernel)
        if (kernel == NLF_LAPLACE2D) {
            wf[j] = 2.0 * inv2pid * p->w_host[m] / kmag;
            gk[j] = std::exp(-0.5 * p->sigma * p->sigma * kk);
        } else if (kernel == NLF_CONFINED2D) {
            // symbol x Jacobian of the confined kernel (Eq. '2Dw1')
            wf[j] = 2.0 * inv2pid * p->w_host[m] * p->st2 * erfcx_host(p->eps * kmag / std::sqrt(2.0));
        } else {
            wf[j] = 2.0 * inv2pid * p->w_host[m] * p->st2;
        }
        // ball of a split evaluation: the partition p(k) = exp(-|k|^2 / a) rides on the weight
        if (p->pweight_a > 0) wf[j] *= std::exp(-kk / p->pweight_a);
    }

    // ---- device buffers ------------------------------------------------------------------------
    const size_t es = elem_size(p->prec);
    // The type-1 output is divided by the Gaussian's Fourier coefficients, up to ~e^{pi msp/4} larger
    // at the corners of the box than at its centre, so FP32 rounding of the inverse transform is
    // amplified; and the dense centre of the spreading grid receives many FP32 atomic additions.
    // FP32 plans with output-driven spreading therefore keep the spreading grid and the inverse FFT
    // in FP64 (node values, the type-2 side and the interpolation stay FP32).
    p->t1_prec = (p->prec == NLF_F32 && (p->use_gather || p->gather_impl_ok)) ? NLF_F64 : p->prec;
    NLF_TRY(dev_alloc(p, &p->grid_a, (size_t)p->batch * p->G * es));
    NLF_TRY(dev_alloc(p, &p->grid_b, (size_t)p->batch * p->G * elem_size(p->t1_prec)));
    NLF_HIP(hipMemsetAsync(p->grid_b, 0, (size_t)p->batch * p->G * elem_size(p->t1_prec), p->stream));
    NLF_TRY(dev_alloc(p, &p->cbuf, (size_t)p->batch * Mh * es));
    if (p->use_gather && p->dim == 3) NLF_TRY(dev_alloc(p, (void**)&p->iacc, (size_t)p->batch * Mh * 2 * sizeof(double)));
    for (int i = 0; i < p->dim; ++i) NLF_TRY(upload(p, (void**)&p->s[i], ss[i].data(), Mh * sizeof(double)));
    // the spreading's per-node tile weights (128 bytes per node): the node positions are fixed
    if ((p->use_gather || p->gather_impl_ok) && weight_table_fits(p)) NLF_TRY(build_weight_table(p));
    NLF_TRY(upload(p, (void**)&p->wfac, wf.data(), Mh * sizeof(double)));
    if (kernel == NLF_LAPLACE2D) NLF_TRY(upload(p, (void**)&p->gk, gk.data(), Mh * sizeof(double)));
    NLF_TRY(upload(p, (void**)&p->perm, order.data(), Mh * sizeof(int)));
    NLF_TRY(upload(p, (void**)&p->chunks, chunks.data(), chunks.size() * sizeof(Chunk)));
    NLF_TRY(build_interp_table(p));   // 2D: the interpolation's per-node start weights (128 bytes per node)
    for (int i = 0; i < p->dim; ++i) {
        // 1 / c_g(j') with c_g(j') = sqrt(tau/pi) exp(-tau j'^2): the Fourier coefficients of the
        // periodised Gaussian exp(-x^2/(4 tau)), tau = pi msp / (3 n^2)
        double tau = pi * p->msp / (3.0 * (double)p->n[i] * p->n[i]);
        std::vector<double> d(p->n[i]);
        for (int j = 0; j < p->n[i]; ++j) {
            double jc = j - p->n[i] / 2;
            d[j] = std::sqrt(pi / tau) * std::exp(tau * jc * jc);
        }
        NLF_TRY(upload(p, (void**)&p->dec[i], d.data(), d.size() * sizeof(double)));
        if (p->prec == NLF_F64) {
            NLF_TRY(upload_twiddles<double>(p, &p->tw_big[i], p->Mr[i]));
            NLF_TRY(upload_twiddles<double>(p, &p->tw_small[i], p->n[i]));
        } else {
            NLF_TRY(upload_twiddles<float>(p, &p->tw_big[i], p->Mr[i]));
            NLF_TRY(upload_twiddles<float>(p, &p->tw_small[i], p->n[i]));
        }
        if (p->t1_prec == p->prec) p->tw_t1[i] = p->tw_big[i];
        else NLF_TRY(upload_twiddles<double>(p, &p->tw_t1[i], p->Mr[i]));
    }
    NLF_TRY(dev_alloc(p, (void**)&p->mom, (size_t)p->batch * 4 * sizeof(double)));
    if (kernel == NLF_LAPLACE2D) {
        // u_{1,1}(x) = -(E1(|x|^2/(2 sigma^2)) + 2 ln|x|) / (4 pi), (gamma_e - ln 2 sigma^2)/(4 pi) at 0
        // (Sec. 2.2, Eq. 'phi1_exct'), written as -(E1(z) + ln z + ln 2 sigma^2)/(4 pi), smooth at 0
        std::vector<double> u(p->N);
        const long double s2 = (long double)p->sigma * p->sigma;
        const long double ln2s2 = logl(2.0L * s2);
        const long double inv4pi = 1.0L / (4.0L * 3.141592653589793238462643383279502884L);
        for (int j0 = 0; j0 < p->n[0]; ++j0)
            for (int j1 = 0; j1 < p->n[1]; ++j1) {
                long double x = -(long double)p->L[0] + j0 * (long double)p->h[0];
                long double y = -(long double)p->L[1] + j1 * (long double)p->h[1];
                long double z = (x * x + y * y) / (2.0L * s2);
                u[(size_t)j0 * p->n[1] + j1] = (double)(-inv4pi * (e1_plus_log(z) + ln2s2));
            }
        NLF_TRY(upload(p, (void**)&p->u11, u.data(), u.size() * sizeof(double)));
    }
    p->red_bytes = (size_t)p->batch * 1024 * 8 * sizeof(double);
    NLF_TRY(dev_alloc(p, (void**)&p->red, p->red_bytes));
    NLF_TRY(dev_alloc(p, (void**)&p->nf_flag, sizeof(int)));
    NLF_HIP(hipMemsetAsync(p->nf_flag, 0, sizeof(int), p->stream));
    return NLF_OK;
}

static int plan_create(const nlf_box* box, int kernel, const nlf_opts* opts, void* stream, double pweight_a,
                       nlf_plan** out) {
    *out = nullptr;
    nlf_plan* p = new (std::nothrow) nlf_plan();
    if (!p) return set_error(NLF_ENOMEM, "host allocation of the plan failed");
    p->stream = (hipStream_t)stream;
    p->box_copy = *box;
    if (opts) p->opts_copy = *opts;
    p->pweight_a = pweight_a;
    int st;
    try {
        st = build(p, box, kernel, opts);
    } catch (const std::bad_alloc&) {
        st = set_error(NLF_ENOMEM, "host allocation failed while building the plan");
    } catch (...) {
        st = set_error(NLF_EINVAL, "unexpected failure while building the plan");
    }
    if (st != NLF_OK) {
        if (p->sub) nlf_plan_destroy(p->sub);
        for (void* q : p->owned) (void)hipFree(q);
        delete p;
        return st;
    }
    *out = p;
    return NLF_OK;
}

static int next_event(nlf_plan* p, size_t* idx) {
    if (p->ev_used == p->ev_pool.size()) {
        hipEvent_t e;
        NLF_HIP(hipEventCreate(&e));
        p->ev_pool.push_back(e);
    }
    *idx = p->ev_used++;
    return NLF_OK;
}

int stage_begin(nlf_plan* p) {
    if (!p->profiling) return -1;
    size_t i;
    if (next_event(p, &i) != NLF_OK) return -1;
    if (hipEventRecord(p->ev_pool[i], p->stream) != hipSuccess) return -1;
    return (int)i;
}

int stage_end(nlf_plan* p, int stage, int mark) {
    if (!p->profiling || mark < 0) return NLF_OK;
    size_t j;
    NLF_TRY(next_event(p, &j));
    NLF_HIP(hipEventRecord(p->ev_pool[j], p->stream));
    p->ev_marks.push_back({stage, {(size_t)mark, j}});
    return NLF_OK;
}

static int drain_events(nlf_plan* p) {
    if (p->ev_marks.empty()) { p->ev_used = 0; return NLF_OK; }
    NLF_HIP(hipStreamSynchronize(p->stream));
    for (auto& m : p->ev_marks) {
        float ms = 0;
        NLF_HIP(hipEventElapsedTime(&ms, p->ev_pool[m.second.first], p->ev_pool[m.second.second]));
        p->stage_ms[m.first] += ms;
        p->stage_cnt[m.first] += 1;
    }
    p->ev_marks.clear();
    p->ev_used = 0;
    return NLF_OK;
}

}  // namespace nlf

using namespace nlf;

extern "C" {

int nlf_plan_create(const nlf_box* box, int kernel, const nlf_opts* opts, void* stream, nlf_plan** out) {
    clear_error();
    if (!box || !out) return set_error(NLF_EINVAL, "box and out must not be NULL");
    return plan_create(box, kernel, opts, stream, 0.0, out);
}

int nlf_plan_set_profiling(nlf_plan* p, int on) {
    clear_error();
    if (!p) return set_error(NLF_EINVAL, "plan must not be NULL");
    if (!on) NLF_TRY(drain_events(p));
    p->profiling = on ? 1 : 0;
    if (p->sub) return nlf_plan_set_profiling(p->sub, on);
    return NLF_OK;
}

int nlf_plan_stage_times(nlf_plan* p, double* ms, long long* counts, int reset) {
    clear_error();
    if (!p) return set_error(NLF_EINVAL, "plan must not be NULL");
    NLF_TRY(drain_events(p));
    double sms[NLF_NSTAGES] = {0};
    long long scnt[NLF_NSTAGES] = {0};
    if (p->sub) NLF_TRY(nlf_plan_stage_times(p->sub, sms, scnt, reset));   // the ball of a split
    for (int i = 0; i < NLF_NSTAGES; ++i) {
        if (ms) ms[i] = p->stage_ms[i] + sms[i];
        if (counts) counts[i] = p->stage_cnt[i] + scnt[i];
        if (reset) { p->stage_ms[i] = 0; p->stage_cnt[i] = 0; }
    }
    return NLF_OK;
}

int nlf_plan_destroy(nlf_plan* p) {
    clear_error();
    if (!p) return NLF_OK;
    (void)hipStreamSynchronize(p->stream);
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    if (p->sws && p->sws_free) p->sws_free(p->sws);
    if (p->twin) nlf_plan_destroy(p->twin);
    if (p->sub) nlf_plan_destroy(p->sub);
    if (p->own_stream) {
        (void)hipStreamSynchronize(p->own_stream);
        (void)hipStreamDestroy(p->own_stream);
    }
    for (void* q : p->owned) (void)hipFree(q);
    delete p;
    return NLF_OK;
}

int nlf_plan_get_info(const nlf_plan* p, nlf_plan_info* info) {
    clear_error();
    if (!p || !info) return set_error(NLF_EINVAL, "plan and info must not be NULL");
    std::memset(info, 0, sizeof *info);
    info->dim = p->dim;
    info->kernel = p->kernel;
    info->prec = p->prec;
    info->batch = p->batch;
    info->msp = p->msp;
    for (int i = 0; i < 3; ++i) {
        info->n[i] = p->n[i];
        info->L[i] = p->L[i];
        info->h[i] = p->h[i];
    }
    info->P = p->P;
    info->sigma = p->sigma;
    info->eps = p->eps;
    info->n_grid = p->N;
    info->n_nodes = p->M;
    info->n_half = p->Mh;
    info->workspace_bytes = p->workspace_bytes;
    info->spread_mode = p->spread_mode;
    info->spread_block = p->spread_kc;
    info->spread_item = p->item_cap;
    info->gather_available = p->use_gather;
    info->bins_available = p->gather_impl_ok;
    info->deterministic = p->deterministic;
    if (p->sub) {
        info->split = 1;
        info->split_a = p->split_a;
        info->split_P2 = p->split_P2;
        info->msp = p->sub->msp;
        info->spread_mode = p->sub->spread_mode;
        info->spread_block = p->sub->spread_kc;
        info->spread_item = p->sub->item_cap;
        info->gather_available = p->sub->use_gather;
        info->bins_available = p->sub->gather_impl_ok;
        info->workspace_bytes += p->sub->workspace_bytes;
    }
    return NLF_OK;
}

int nlf_plan_nodes(const nlf_plan* p, double* k_host, double* w_host) {
    clear_error();
    if (!p) return set_error(NLF_EINVAL, "plan must not be NULL");
    if (p->sub) return nlf_plan_nodes(p->sub, k_host, w_host);   // the ball of a split
    if (k_host) std::memcpy(k_host, p->k_host.data(), p->k_host.size() * sizeof(double));
    if (w_host) std::memcpy(w_host, p->w_host.data(), p->w_host.size() * sizeof(double));
    return NLF_OK;
}

const char* nlf_last_error(void) { return nlf::g_err; }

const char* nlf_strerror(int s) {
    switch (s) {
        case NLF_OK: return "ok";
        case NLF_EINVAL: return "invalid argument";
        case NLF_EUNSUPPORTED: return "unsupported configuration";
        case NLF_ENOMEM: return "out of memory";
        case NLF_EHIP: return "HIP runtime error";
        case NLF_ENOCONV: return "iteration cap reached without convergence";
        case NLF_ENONFINITE: return "non-finite value detected";
        default: return "unknown status";
    }
}

const char* nlf_version(void) { return "nlf 0.1 (gfx950)"; }

}  // extern "C"
