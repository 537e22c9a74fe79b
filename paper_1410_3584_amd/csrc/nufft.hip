// NUFFT stages of the potential evaluation on gfx950 (Sec. 2.1, Eq. 'ifft'; Sec. 2.2, Alg. 1).
//
// Gaussian gridding with oversampling 2: a node at position s (in oversampled cells) couples to
// the 2*msp cells l0+p, p = -msp+1..msp, l0 = floor(s), with the separable weight
// prod_i exp(-alpha (p_i - delta_i)^2), delta_i = s_i - l0_i.
//
// Main path (tile-gathered, FP64 matrix cores).  The oversampled grid is cut into gather tiles of
// 8 x 16 cells (2D) or 8 x 4 x 4 cells (3D); the plan lists, per tile, the nodes whose stencil
// overlaps it, in items of <= kMChunk nodes.  For one item both directions are dense products:
//   spreading (type-1):      F = A^T B, A[k][(comp, x)] = c_k w0_k[x], B[k][j] = tile weights
//   interpolation (type-2):  H = G B,   then u_k = sum_x w0_k[x] H[x][k]
// computed with v_mfma_f64_16x16x4 from weights staged in LDS; tiles receive their sums with
// one atomic per cell component, nodes with one per component and tile.  The symbol/weight
// multiply (the symbol_weight step) is the per-node epilogue of the interpolation, in FP64.
// 2D interpolation works per bin of nodes instead (k_binterp2): the bin's grid window in LDS is
// the A operand and the nodes' weights the B operand, with no atomics.
// Fallback (candidate list too large, 3D): node-parallel kernels over binned chunks, the grid
// window staged in LDS (interpolation) or LDS atomics (spreading).
// Only half of the node set is evaluated: rho is real, so rhohat(-k) = conj(rhohat(k)), and the
// node set is symmetric under k -> -k (even n_phi, symmetric Gauss-Legendre in cos theta).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "nufft_dev.h"

namespace nlf {

// ---- host side ---------------------------------------------------------------------------------
static NodeArgs node_args(const nlf_plan* p) {
    NodeArgs na{};
    na.dim = p->dim;
    for (int i = 0; i < 3; ++i) {
        na.Mr[i] = p->Mr[i];
        na.tile[i] = p->tile[i];
        na.W[i] = p->window[i];
        na.s[i] = p->s[i];
    }
    na.chunks = p->chunks;
    na.nchunks = p->nchunks;
    na.gc = p->gc;
    na.csplit = p->chunk_split;
    na.isplit = p->item_split;
    na.wtab = reinterpret_cast<const double2*>(p->wtab);
    na.itab = reinterpret_cast<const double2*>(p->itab);
    return na;
}

// The weight table of a 2D plan (see NodeArgs::wtab): for sorted node m and axis i, the gather
// tiles (GT_0 = 8, GT_1 = 16 cells) from the one holding the stencil's first cell l0 - msp + 1 on,
// four of them, each stored at slot (tile index mod 4).  A stencil overlaps at most four
// consecutive tiles, so every tile whose candidate list holds the node finds its own values.
__global__ void k_weight_table(const double* __restrict__ s0, const double* __restrict__ s1, long long Mh, int Mr0,
                               int Mr1, int msp, double alpha, double2* __restrict__ wt) {
    for (long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x; m < Mh; m += (long long)gridDim.x * blockDim.x) {
#pragma unroll
        for (int ax = 0; ax < 2; ++ax) {
            const double s = ax == 0 ? s0[m] : s1[m];
            const int Mr = ax == 0 ? Mr0 : Mr1, gt = ax == 0 ? 8 : 16, ng = Mr / gt;
            const int first = wrap((int)floor(s) - msp + 1, Mr) / gt;
            for (int j = 0; j < 4; ++j) {
                const int tl = (first + j) & (ng - 1);
                wt[8 * m + 4 * ax + (tl & 3)] = tile_start(s, tl * gt, Mr, msp, alpha);
            }
        }
    }
}

// The interpolation table of a 2D plan (see NodeArgs::itab), one workgroup per chunk: node t of a
// chunk belongs to the group of 16 starting at t - t mod 16 (the interpolation's wave groups).
template <int MSP, bool F32>
__global__ void k_interp_table(const Chunk* __restrict__ chunks, const double* __restrict__ s0,
                               const double* __restrict__ s1, int Mr0, int Mr1, double alpha, double2* __restrict__ it) {
    const Chunk ch = chunks[blockIdx.x];
    const int t = threadIdx.x;
    if (t >= ch.count) return;
    const int node = ch.start + t, first = ch.start + (t & ~15);
    const double f0 = floor(s0[node]), f1 = floor(s1[node]);
    const int rx0 = wrap((int)f0, Mr0) - ch.t0 * 8, ry0 = wrap((int)f1, Mr1) - ch.t1 * 16;
    const int c0 = wrap((int)floor(s1[first]), Mr1) - ch.t1 * 16;
    for (int ka = 0; ka < 4; ++ka) {
        double2 wy, wx;
        if (F32) binterp2_32_starts<MSP>(s0[node] - f0, s1[node] - f1, rx0, ry0, c0, ka, alpha, wy, wx);
        else binterp2_starts<MSP>(s0[node] - f0, s1[node] - f1, rx0, ry0, c0, ka, alpha, wy, wx);
        it[2 * (4 * (long long)node + ka)] = wy;
        it[2 * (4 * (long long)node + ka) + 1] = wx;
    }
}

template <int MSP, bool F32>
static int interp_table_t(nlf_plan* p) {
    NLF_TRY(dev_alloc(p, &p->itab, (size_t)p->Mh * 8 * sizeof(double2)));
    hipLaunchKernelGGL((k_interp_table<MSP, F32>), dim3(p->nchunks), dim3(kChunk), 0, p->stream, p->chunks, p->s[0],
                       p->s[1], p->Mr[0], p->Mr[1], p->gc.alpha, reinterpret_cast<double2*>(p->itab));
    NLF_HIP(hipGetLastError());
    return NLF_OK;
}

int build_interp_table(nlf_plan* p) {
    if (p->dim != 2 || p->nchunks == 0) return NLF_OK;
    if (p->prec == NLF_F64) {
        switch (p->msp) {
            case 8: return interp_table_t<8, false>(p);
            case 9: return interp_table_t<9, false>(p);
            case 10: return interp_table_t<10, false>(p);
            case 11: return interp_table_t<11, false>(p);
            case 12: return interp_table_t<12, false>(p);
            case 13: return interp_table_t<13, false>(p);
            case 14: return interp_table_t<14, false>(p);
            case 16: return interp_table_t<16, false>(p);
            default: return NLF_OK;
        }
    }
    switch (p->msp) {
        case 4: return interp_table_t<4, true>(p);
        case 5: return interp_table_t<5, true>(p);
        case 6: return interp_table_t<6, true>(p);
        case 7: return interp_table_t<7, true>(p);
        case 8: return interp_table_t<8, true>(p);
        case 9: return interp_table_t<9, true>(p);
        case 10: return interp_table_t<10, true>(p);
        default: return NLF_OK;
    }
}

bool weight_table_fits(const nlf_plan* p) {
    // every tile a stencil overlaps has a slot (at most 4 along each axis: msp <= 12), the tile
    // counts are multiples of 4 (slots agree across the periodic wrap), and tile_start() applies
    return p->dim == 2 && p->msp <= 12 && p->Mr[0] % 32 == 0 && p->Mr[1] % 64 == 0 &&
           p->Mr[0] >= 2 * p->msp + 8 && p->Mr[1] >= 2 * p->msp + 16;
}

int build_weight_table(nlf_plan* p) {
    NLF_TRY(dev_alloc(p, &p->wtab, (size_t)p->Mh * 8 * sizeof(double2)));
    dim3 grid((unsigned)std::min<long long>((p->Mh + 255) / 256, 4096));
    hipLaunchKernelGGL(k_weight_table, grid, dim3(256), 0, p->stream, p->s[0], p->s[1], p->Mh, p->Mr[0], p->Mr[1],
                       p->msp, p->gc.alpha, reinterpret_cast<double2*>(p->wtab));
    NLF_HIP(hipGetLastError());
    return NLF_OK;
}

static size_t window_bytes(const nlf_plan* p) {
    size_t e = elem_size(p->prec);
    return (p->dim == 2) ? (size_t)p->window[0] * p->window[1] * e : (size_t)p->window[1] * p->window[2] * e;
}

static int grid_chunks(const nlf_plan* p) { return ((p->nchunks + 7) / 8) * 8; }

template <typename T, int MSP>
static int interp_t(nlf_plan* p, const EpiArgs& ea, bool zero_b) {
    NodeArgs na = node_args(p);
    if (p->dim == 2) {
        dim3 grid(8 * p->chunk_split.per, p->batch);
        const double qq4 = exp(-32.0 * p->gc.alpha);
        const size_t bbytes = (size_t)p->batch * p->G * elem_size(p->t1_prec);   // a multiple of 16
        double2* zb = zero_b ? (double2*)p->grid_b : nullptr;
        if (Recorder* rec = recorder()) {   // the persistent executor's bodies: default widths
            constexpr bool d = std::is_same<T, double>::value;
            if (MSP != (d ? 12 : 7)) {
                rec->failed = 1;
                return NLF_OK;
            }
            BinterpTask t{p->grid_a, p->G, na, ea, qq4, exp(-2.0 * p->gc.alpha), zb, (long long)(bbytes / 16)};
            return record(rec, d ? TK_BINTERP_D : TK_BINTERP_F, grid, 0, t);
        }
        if constexpr (std::is_same<T, float>::value) {   // FP32 plans: the FP32 matrix cores
            if (p->itab)
                hipLaunchKernelGGL((k_binterp2_32<MSP, true>), grid, dim3(256), 0, p->stream,
                                   reinterpret_cast<const float2*>(p->grid_a), p->G, na, ea, qq4,
                                   exp(-2.0 * p->gc.alpha), zb, (long long)(bbytes / 16));
            else
                hipLaunchKernelGGL((k_binterp2_32<MSP, false>), grid, dim3(256), 0, p->stream,
                                   reinterpret_cast<const float2*>(p->grid_a), p->G, na, ea, qq4,
                                   exp(-2.0 * p->gc.alpha), zb, (long long)(bbytes / 16));
        } else if (p->itab) {
            hipLaunchKernelGGL((k_binterp2<T, MSP, true>), grid, dim3(256), 0, p->stream,
                               reinterpret_cast<const V2<T>*>(p->grid_a), p->G, na, ea, qq4, zb,
                               (long long)(bbytes / 16));
        } else {
            hipLaunchKernelGGL((k_binterp2<T, MSP, false>), grid, dim3(256), 0, p->stream,
                               reinterpret_cast<const V2<T>*>(p->grid_a), p->G, na, ea, qq4, zb,
                               (long long)(bbytes / 16));
        }
        NLF_HIP(hipGetLastError());
        return NLF_OK;
    }
    // (the tile-gathered 3D interpolation reads the explicit candidate lists through the work
    // items; with neighbour-bin items in use, or on a deterministic plan, whose sums must not go
    // through atomics, it takes the plane-streamed kernel)
    if (p->use_gather && !p->items_bins && !p->deterministic) {
        NLF_TRY(fill_zero(p, p->iacc, (size_t)p->batch * p->Mh * 2 * sizeof(double)));
        dim3 ggrid(8 * p->item_split.per, p->batch);
        const double qq = exp(-2.0 * p->gc.alpha);
        const V2<T>* g = reinterpret_cast<const V2<T>*>(p->grid_a);
        if (p->dim == 2)
            hipLaunchKernelGGL((k_minterp<T, MSP, 2>), ggrid, dim3(2 * kMChunk), 0, p->stream, g, p->G,
                               (double2*)p->iacc, p->Mh, na, p->gitems, p->ngitems, p->gcand, qq);
        else
            hipLaunchKernelGGL((k_minterp<T, MSP, 3>), ggrid, dim3(2 * kMChunk), 0, p->stream, g, p->G,
                               (double2*)p->iacc, p->Mh, na, p->gitems, p->ngitems, p->gcand, qq);
        NLF_HIP(hipGetLastError());
        dim3 egrid((unsigned)std::min<long long>((p->Mh + 255) / 256, 4096), p->batch);
        hipLaunchKernelGGL((k_iepilogue<T>), egrid, dim3(256), 0, p->stream, (const double2*)p->iacc, p->Mh, p->Mh,
                           na, ea);
        NLF_HIP(hipGetLastError());
        return NLF_OK;
    }
    dim3 grid(grid_chunks(p), p->batch);
    const V2<T>* g = reinterpret_cast<const V2<T>*>(p->grid_a);
    hipLaunchKernelGGL((k_interp3<T, MSP>), grid, dim3(kChunk), window_bytes(p), p->stream, g, p->G, na, ea);
    NLF_HIP(hipGetLastError());
    return NLF_OK;
}

template <typename T, int MSP, int KC, bool BINS>
static int gather_spread_t(nlf_plan* p) {
    NodeArgs na = node_args(p);
    V2<T>* g = reinterpret_cast<V2<T>*>(p->grid_b);
    const V2<T>* c = reinterpret_cast<const V2<T>*>(p->cbuf);
    dim3 ggrid(8 * p->item_split.per, p->batch);
    const double qq = exp(-2.0 * p->gc.alpha);
    BinArgs ba{};
    ba.bin_off = p->bin_off;
    for (int i = 0; i < 3; ++i) {
        ba.lo[i] = p->impl_lo[i];
        ba.n[i] = p->impl_n[i];
        ba.NB[i] = p->gng[i];
    }
    // deterministic plans: the items of tiles of several store partial sums, added in order below
    double* pscr = (p->deterministic && p->ntred > 0) ? p->pscratch : nullptr;
    const long long sstride = p->nslots * 256;
    if (Recorder* rec = recorder()) {   // the persistent executor's bodies: 2D lists, 128-candidate blocks
        constexpr bool d = std::is_same<T, double>::value;
        const bool ok = p->dim == 2 && KC == 128 && !BINS && !pscr && MSP == (d ? 12 : 7) &&
                        (d ? p->t1_prec == NLF_F64 : p->t1_prec == NLF_F64);
        if (!ok) {
            rec->failed = 1;
            return NLF_OK;
        }
        MspreadTask t{p->grid_b, p->G, p->cbuf, p->Mh, na, p->gitems, p->ngitems, p->gcand, qq, ba};
        return record(rec, d ? TK_MSPREAD_D : TK_MSPREAD_F, ggrid, 0, t);
    }
    bool done = false;
    if constexpr (std::is_same<T, float>::value) {
        if (p->t1_prec != p->prec) {   // FP32 node values: FP32 matrix cores, FP64 spreading grid
            double2* g64 = reinterpret_cast<double2*>(p->grid_b);
            if (p->dim == 2 && p->wtab && !BINS)   // explicit lists only, as for FP64 below
                hipLaunchKernelGGL((k_mspread32<MSP, 2, KC, BINS, !BINS>), ggrid, dim3(2 * KC), 0, p->stream, g64,
                                   p->G, c, p->Mh, na, p->gitems, p->ngitems, p->gcand, qq, ba, pscr, sstride);
            else if (p->dim == 2)
                hipLaunchKernelGGL((k_mspread32<MSP, 2, KC, BINS, false>), ggrid, dim3(2 * KC), 0, p->stream, g64,
                                   p->G, c, p->Mh, na, p->gitems, p->ngitems, p->gcand, qq, ba, pscr, sstride);
            else
                hipLaunchKernelGGL((k_mspread32<MSP, 3, KC, BINS, false>), ggrid, dim3(2 * KC), 0, p->stream, g64,
                                   p->G, c, p->Mh, na, p->gitems, p->ngitems, p->gcand, qq, ba, pscr, sstride);
            done = true;
        }
    }
    if (done) {
    } else if (p->dim == 2) {
        // the table holds the tiles of the explicit lists (at most 4 per axis); the neighbour-bin
        // streams also pass nodes of the bins next to those, which need the Gaussian's tail
        constexpr bool kTab = MSP <= 12 && !BINS;   // the widths weight_table_fits() admits
        bool launched = false;
        if constexpr (kTab) {
            if (p->wtab) {
                hipLaunchKernelGGL((k_mspread<T, T, MSP, 2, KC, BINS, true>), ggrid, dim3(2 * KC), 0, p->stream, g,
                                   p->G, c, p->Mh, na, p->gitems, p->ngitems, p->gcand, qq, ba, pscr, sstride);
                launched = true;
            }
        }
        if (!launched)
            hipLaunchKernelGGL((k_mspread<T, T, MSP, 2, KC, BINS, false>), ggrid, dim3(2 * KC), 0, p->stream, g, p->G,
                               c, p->Mh, na, p->gitems, p->ngitems, p->gcand, qq, ba, pscr, sstride);
    } else {
        hipLaunchKernelGGL((k_mspread<T, T, MSP, 3, KC, BINS, false>), ggrid, dim3(2 * KC), 0, p->stream, g, p->G, c,
                           p->Mh, na, p->gitems, p->ngitems, p->gcand, qq, ba, pscr, sstride);
    }
    NLF_HIP(hipGetLastError());
    if (pscr) {
        const dim3 rgrid(p->ntred, p->batch);
        if (p->t1_prec != p->prec) {
            double2* g64 = reinterpret_cast<double2*>(p->grid_b);
            if (p->dim == 2)
                hipLaunchKernelGGL((k_tile_reduce<double, 2>), rgrid, dim3(256), 0, p->stream, g64, p->G, pscr, sstride,
                                   p->tred, na);
            else
                hipLaunchKernelGGL((k_tile_reduce<double, 3>), rgrid, dim3(256), 0, p->stream, g64, p->G, pscr, sstride,
                                   p->tred, na);
        } else if (p->dim == 2) {
            hipLaunchKernelGGL((k_tile_reduce<T, 2>), rgrid, dim3(256), 0, p->stream, g, p->G, pscr, sstride, p->tred, na);
        } else {
            hipLaunchKernelGGL((k_tile_reduce<T, 3>), rgrid, dim3(256), 0, p->stream, g, p->G, pscr, sstride, p->tred, na);
        }
        NLF_HIP(hipGetLastError());
    }
    return NLF_OK;
}

template <typename T, int MSP>
static int spread_t(nlf_plan* p) {
    if (p->use_gather && p->spread_mode == NLF_SPREAD_GATHER)
        return p->spread_kc == 128 ? gather_spread_t<T, MSP, 128, false>(p) : gather_spread_t<T, MSP, 64, false>(p);
    if (p->gather_impl_ok && p->spread_mode == NLF_SPREAD_BINS)
        return p->spread_kc == 128 ? gather_spread_t<T, MSP, 128, true>(p) : gather_spread_t<T, MSP, 64, true>(p);
    NodeArgs na = node_args(p);
    V2<T>* g = reinterpret_cast<V2<T>*>(p->grid_b);
    const V2<T>* c = reinterpret_cast<const V2<T>*>(p->cbuf);
    dim3 grid(grid_chunks(p), p->batch);
    if (p->dim == 2)
        hipLaunchKernelGGL((k_spread2<T, MSP>), grid, dim3(kChunk), window_bytes(p), p->stream, g, p->G, c, p->Mh, na);
    else
        hipLaunchKernelGGL((k_spread3<T, MSP>), grid, dim3(kChunk), window_bytes(p), p->stream, g, p->G, c, p->Mh, na);
    NLF_HIP(hipGetLastError());
    return NLF_OK;
}

// msp dispatch: FP64 plans use msp in [8, 16], FP32 plans msp in [4, 10]
#define NLF_MSP_CASES_F64(F, T, ...) \
    case 8: return F<T, 8>(__VA_ARGS__); case 9: return F<T, 9>(__VA_ARGS__); \
    case 10: return F<T, 10>(__VA_ARGS__); case 11: return F<T, 11>(__VA_ARGS__); \
    case 12: return F<T, 12>(__VA_ARGS__); case 13: return F<T, 13>(__VA_ARGS__); \
    case 14: return F<T, 14>(__VA_ARGS__); case 16: return F<T, 16>(__VA_ARGS__);
#define NLF_MSP_CASES_F32(F, T, ...) \
    case 4: return F<T, 4>(__VA_ARGS__); case 5: return F<T, 5>(__VA_ARGS__); \
    case 6: return F<T, 6>(__VA_ARGS__); case 7: return F<T, 7>(__VA_ARGS__); \
    case 8: return F<T, 8>(__VA_ARGS__); case 9: return F<T, 9>(__VA_ARGS__); \
    case 10: return F<T, 10>(__VA_ARGS__);

static int bad_msp(const nlf_plan* p) {
    return set_error(NLF_EUNSUPPORTED, "msp = %d has no compiled kernel for this precision "
                     "(FP64: 8-14, 16; FP32: 4-10)", p->msp);
}

static EpiArgs epi_args(const nlf_plan* p, int mode, void* out, long long ostride) {
    EpiArgs ea{};
    ea.mode = mode;
    ea.out = out;
    ea.ostride = ostride;
    ea.wfac = p->wfac;
    ea.gk = p->gk;
    ea.mom = p->mom;
    ea.st2 = p->st2;
    for (int i = 0; i < 3; ++i) ea.kscale[i] = (i < p->dim) ? 3.14159265358979323846 / (2.0 * p->L[i]) : 0.0;
    ea.perm = p->perm;
    ea.hphi = p->n_phi / 2;
    ea.n_phi = p->n_phi;
    ea.n_theta = p->n_theta;
    return ea;
}

int interp(nlf_plan* p, int mode, void* out, bool zero_b) {
    EpiArgs ea;
    if (mode == MODE_TYPE2) ea = epi_args(p, MODE_TYPE2, out, p->M);
    else ea = epi_args(p, p->kernel == NLF_LAPLACE2D ? MODE_LAPLACE : MODE_COULOMB, p->cbuf, p->Mh);
    if (p->prec == NLF_F64) {
        switch (p->msp) { NLF_MSP_CASES_F64(interp_t, double, p, ea, zero_b) default: return bad_msp(p); }
    }
    switch (p->msp) { NLF_MSP_CASES_F32(interp_t, float, p, ea, zero_b) default: return bad_msp(p); }
}

static int spread_only(nlf_plan* p) {
    if (p->prec == NLF_F64) {
        switch (p->msp) { NLF_MSP_CASES_F64(spread_t, double, p) default: return bad_msp(p); }
    }
    switch (p->msp) { NLF_MSP_CASES_F32(spread_t, float, p) default: return bad_msp(p); }
}

int spread(nlf_plan* p) {
    NLF_TRY(fill_zero(p, p->grid_b, (size_t)p->batch * p->G * elem_size(p->t1_prec)));
    return spread_only(p);
}

int fold_c(nlf_plan* p, const void* c) {
    dim3 grid((unsigned)std::min<long long>((p->Mh + 255) / 256, 4096), p->batch);
    if (p->prec == NLF_F64)
        hipLaunchKernelGGL((k_fold<double>), grid, dim3(256), 0, p->stream, (const double2*)c, p->M,
                           (double2*)p->cbuf, p->Mh, p->perm, p->n_phi / 2, p->n_phi, p->n_theta);
    else
        hipLaunchKernelGGL((k_fold<float>), grid, dim3(256), 0, p->stream, (const float2*)c, p->M,
                           (float2*)p->cbuf, p->Mh, p->perm, p->n_phi / 2, p->n_phi, p->n_theta);
    NLF_HIP(hipGetLastError());
    return NLF_OK;
}

#define NLF_STAGE(p, id, call)               \
    do {                                     \
        int mk_ = stage_begin(p);            \
        NLF_TRY(call);                       \
        NLF_TRY(stage_end(p, id, mk_));      \
    } while (0)

// the band cube |f_i| < band of the spreading grid of a split's ball (the only cells spread into)
template <typename T>
__global__ void k_zero_band(V2<T>* __restrict__ grid, long long G, int band, int Mr1, int Mr2, int Mr0) {
    V2<T>* g = grid + (long long)blockIdx.y * G;
    const int w = 2 * band;
    const long long cnt = (long long)w * w * w;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (long long)gridDim.x * blockDim.x) {
        const int i0 = (int)(i / ((long long)w * w)), r = (int)(i - (long long)i0 * w * w);
        const int i1 = r / w, i2 = r - i1 * w;
        const int c0 = i0 < band ? i0 : Mr0 - w + i0;
        const int c1 = i1 < band ? i1 : Mr1 - w + i1;
        const int c2 = i2 < band ? i2 : Mr2 - w + i2;
        g[((long long)c0 * Mr1 + c1) * Mr2 + c2] = mk2<T>((T)0, (T)0);
    }
}

static int zero_spread_grid(nlf_plan* p) {
    if (!p->band) return fill_zero(p, p->grid_b, (size_t)p->batch * p->G * elem_size(p->t1_prec));
    const long long w = 2LL * p->band;
    dim3 grid((unsigned)std::min<long long>((w * w * w + 255) / 256, 8192), p->batch);
    if (p->t1_prec == NLF_F64)
        hipLaunchKernelGGL((k_zero_band<double>), grid, dim3(256), 0, p->stream, (double2*)p->grid_b, p->G, p->band,
                           p->Mr[1], p->Mr[2], p->Mr[0]);
    else
        hipLaunchKernelGGL((k_zero_band<float>), grid, dim3(256), 0, p->stream, (float2*)p->grid_b, p->G, p->band,
                           p->Mr[1], p->Mr[2], p->Mr[0]);
    NLF_HIP(hipGetLastError());
    return NLF_OK;
}

int potential(nlf_plan* p, const void* rho, void* u) {
    if (p->sub) {
        // split (Eq. '3.9'): I2 by the ball plan writes u, then I1 = the cyclic convolution of the
        // padded density with w adds to it; the ball plan follows this plan's current stream
        p->sub->stream = p->stream;
        NLF_TRY(potential(p->sub, rho, u));
        NLF_STAGE(p, NLF_STAGE_FFT_INV, fft_split_i1(p, rho, u));
        return NLF_OK;
    }
    const bool lap = p->kernel == NLF_LAPLACE2D;   // moments m0, m1: computed by the forward FFT
    NLF_STAGE(p, NLF_STAGE_FFT_FWD, fft_type2_forward(p, rho));
    // 2D: the interpolation kernel also clears the spreading grid (the zero stage then reports 0)
    const bool fused_zero = (p->dim == 2);
    NLF_STAGE(p, NLF_STAGE_INTERP, interp(p, 0, nullptr, fused_zero));
    if (!fused_zero) NLF_STAGE(p, NLF_STAGE_ZERO, zero_spread_grid(p));
    NLF_STAGE(p, NLF_STAGE_SPREAD, spread_only(p));
    NLF_STAGE(p, NLF_STAGE_FFT_INV, fft_type1_inverse(p, u, lap));
    return NLF_OK;
}

}  // namespace nlf

using namespace nlf;

extern "C" {

// check_finite plans: the flag is cleared before the call's work (a solver may have left it set)
// and read, with a stream synchronisation, after it
static int finite_begin(nlf_plan* p) {
    if (!p->check_finite) return NLF_OK;
    int seen = 0;
    return read_nonfinite(p, &seen);
}
static int finite_end(nlf_plan* p) {
    if (!p->check_finite) return NLF_OK;
    int seen = 0;
    NLF_TRY(read_nonfinite(p, &seen));
    if (seen) return set_error(NLF_ENONFINITE, "the density holds a NaN or Inf value");
    return NLF_OK;
}

int nlf_potential(nlf_plan* p, const void* rho, void* u) {
    clear_error();
    if (!p || !rho || !u) return set_error(NLF_EINVAL, "plan, rho and u must not be NULL");
    if (rho == u) return set_error(NLF_EINVAL, "rho and u may not alias");
    NLF_TRY(finite_begin(p));
    NLF_TRY(potential(p, rho, u));
    return finite_end(p);
}

int nlf_type2(nlf_plan* p, const void* rho, void* rhohat) {
    clear_error();
    if (!p || !rho || !rhohat) return set_error(NLF_EINVAL, "plan, rho and rhohat must not be NULL");
    NLF_TRY(finite_begin(p));
    if (p->sub) {   // the ball of a split
        p->sub->stream = p->stream;
        NLF_TRY(fft_type2_forward(p->sub, rho));
        NLF_TRY(interp(p->sub, MODE_TYPE2, rhohat, false));
    } else {
        NLF_TRY(fft_type2_forward(p, rho));
        NLF_TRY(interp(p, MODE_TYPE2, rhohat, false));
    }
    return finite_end(p);
}

int nlf_type1(nlf_plan* p, const void* c, void* u) {
    clear_error();
    if (!p || !c || !u) return set_error(NLF_EINVAL, "plan, c and u must not be NULL");
    if (p->sub) {   // the ball of a split
        p->sub->stream = p->stream;
        return nlf_type1(p->sub, c, u);
    }
    NLF_TRY(fold_c(p, c));
    NLF_TRY(spread(p));
    return fft_type1_inverse(p, u, false);
}

int nlf_plan_set_spread(nlf_plan* p, int mode, int block, int item) {
    clear_error();
    if (!p) return set_error(NLF_EINVAL, "plan must not be NULL");
    if (p->sub) return nlf_plan_set_spread(p->sub, mode, block, item);   // the ball of a split
    if (p->deterministic)
        return set_error(NLF_EINVAL, "a deterministic plan keeps its one-item-per-tile spreading");
    if (mode != NLF_SPREAD_GATHER && mode != NLF_SPREAD_SCATTER && mode != NLF_SPREAD_BINS)
        return set_error(NLF_EINVAL, "spread mode must be NLF_SPREAD_GATHER, _SCATTER or _BINS");
    if (mode == NLF_SPREAD_SCATTER) {
        // the scatter kernels accumulate in the plan's precision; FP32 plans keep an FP64
        // spreading grid for the gather kernels (the FP32 bar needs it)
        if (p->t1_prec != p->prec)
            return set_error(NLF_EINVAL, "this plan spreads into an FP64 grid: only the gather modes");
        p->spread_mode = mode;
        return NLF_OK;
    }
    const bool bins = (mode == NLF_SPREAD_BINS);
    if (!bins && !p->use_gather) return set_error(NLF_EINVAL, "this plan has no gather-tile candidate lists");
    if (bins && !p->gather_impl_ok) return set_error(NLF_EINVAL, "the neighbour-bin gather does not apply to this plan");
    if (block != 64 && block != 128) return set_error(NLF_EINVAL, "block must be 64 or 128");
    if (!(item == 512 || item == 1024 || item == 2048 || (item == 256 && !bins)))
        return set_error(NLF_EINVAL, "item must be 256 (lists only), 512, 1024 or 2048");
    if (item != p->item_cap || (p->items_bins != 0) != bins) NLF_TRY(set_items(p, item, bins));
    p->spread_mode = mode;
    p->spread_kc = block;
    return NLF_OK;
}

int nlf_plan_autotune(nlf_plan* p, int reps, double* best_ms) {
    clear_error();
    if (!p) return set_error(NLF_EINVAL, "plan must not be NULL");
    if (p->sub) {   // the ball of a split
        p->sub->stream = p->stream;
        return nlf_plan_autotune(p->sub, reps, best_ms);
    }
    if (reps <= 0) reps = 5;
    struct Cfg { int mode, block, item; };
    std::vector<Cfg> cfgs;
    if (p->deterministic)   // timed, not changed
        cfgs.push_back({p->spread_mode, p->spread_kc, p->item_cap});
    else if (p->use_gather)
        for (int block : {64, 128})
            for (int item : {256, 512, 1024, 2048}) cfgs.push_back({NLF_SPREAD_GATHER, block, item});
    if (p->gather_impl_ok && !p->deterministic)
        for (int block : {64, 128})
            for (int item : {512, 1024, 2048}) cfgs.push_back({NLF_SPREAD_BINS, block, item});
    if (p->t1_prec == p->prec && !p->deterministic) cfgs.push_back({NLF_SPREAD_SCATTER, p->spread_kc, p->item_cap});
    if (cfgs.empty()) return set_error(NLF_EINVAL, "no spreading decomposition to time");
    // node values 1: every tile the candidates reach receives a nonzero sum
    const long long nv = (long long)p->batch * p->Mh;
    if (p->prec == NLF_F64)
        hipLaunchKernelGGL((k_fill_one<double>), dim3((unsigned)std::min<long long>((nv + 255) / 256, 65535)), dim3(256),
                           0, p->stream, (double2*)p->cbuf, nv);
    else
        hipLaunchKernelGGL((k_fill_one<float>), dim3((unsigned)std::min<long long>((nv + 255) / 256, 65535)), dim3(256),
                           0, p->stream, (float2*)p->cbuf, nv);
    NLF_HIP(hipGetLastError());
    hipEvent_t e0, e1;
    NLF_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(NLF_EHIP, "hipEventCreate failed");
    }
    double best = 1e300;
    Cfg bc = cfgs.front();
    int rc = NLF_OK;
    for (const Cfg& c : cfgs) {
        if (!p->deterministic && (rc = nlf_plan_set_spread(p, c.mode, c.block, c.item)) != NLF_OK) break;
        if ((rc = spread_only(p)) != NLF_OK) break;   // warm-up
        if (hipEventRecord(e0, p->stream) != hipSuccess) { rc = set_error(NLF_EHIP, "hipEventRecord failed"); break; }
        for (int r = 0; r < reps && rc == NLF_OK; ++r) rc = spread_only(p);
        if (rc != NLF_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, p->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = set_error(NLF_EHIP, "timing the spreading failed");
            break;
        }
        if (ms / reps < best) {
            best = ms / reps;
            bc = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != NLF_OK) return rc;
    if (!p->deterministic) NLF_TRY(nlf_plan_set_spread(p, bc.mode, bc.block, bc.item));
    if (best_ms) *best_ms = best;
    return NLF_OK;
}

}  // extern "C"
