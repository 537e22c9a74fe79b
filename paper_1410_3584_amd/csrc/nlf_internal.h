// Internal declarations shared by the library's translation units (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

#include "nlf.h"

namespace nlf {

// ---- error state -------------------------------------------------------------------------
int set_error(int code, const char* fmt, ...);
void clear_error();

#define NLF_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::nlf::set_error(NLF_EHIP, "%s failed at %s:%d: %s", #call, __FILE__, \
                                    __LINE__, hipGetErrorString(e_));                   \
    } while (0)

#define NLF_TRY(call)            \
    do {                         \
        int s_ = (call);         \
        if (s_ != NLF_OK) return s_; \
    } while (0)

// ---- small device-side value types ------------------------------------------------------------
template <typename T> struct V2t;
template <> struct V2t<float>  { using type = float2; };
template <> struct V2t<double> { using type = double2; };
template <typename T> using V2 = typename V2t<T>::type;

// A chunk is up to kChunk consecutive sorted nodes that fall in one bin of the oversampled grid.
struct Chunk {
    int start, count;  // first sorted node, number of nodes (<= kChunk)
    int t0, t1, t2;    // bin coordinates (tiles along axes 0,1,2; t2 unused in 2D)
    int pad;
};

constexpr int kChunk = 128;   // threads per interpolation/spreading workgroup = nodes per chunk
constexpr int kMaxMsp = 16;

// A tile-gather work item: up to kMItem candidate nodes of one gather tile of the oversampled
// grid (8 x 16 cells in 2D, 8 x 4 x 4 in 3D: 128 cells), taken kMChunk at a time.
struct GItem {
    int g0, g1, g2;    // tile coordinates
    int count;         // candidates in this item
    long long start;   // first entry in the candidate list
    int only;          // 1: the tile's only item (the spreading stores its sums instead of adding)
    int slot;          // deterministic plans, tiles of several items: the item's partial-sum slot
};
// Deterministic plans: a tile of several work items, whose items store their partial sums in the
// slots [first, first + n) that k_tile_reduce then adds in slot order.
struct TileRed {
    int g0, g1, g2;
    int first, n;
};
constexpr int kMChunk = 128;
constexpr int kMItem = 1024;

// A launch's work list split over the 8 XCDs.  Hardware workgroup ids go round-robin over the XCDs,
// so XCD x runs the workgroups b with b mod 8 = x; it takes the consecutive entries [s[x], s[x+1])
// of the list (neighbouring bins and tiles share its L2), the cuts placed at equal estimated cost
// (the polar nodes crowd the low frequencies, so equal entry counts leave some XCDs with far more
// work).  The launch has 8 per workgroups, per = the longest range.
struct XcdSplit {
    int s[9];
    int per;
};
XcdSplit xcd_split(const std::vector<long long>& cost);
// neighbour-bin gather: most neighbour bins a tile may read (5 x 9 x 9 at msp 16 in 3D)
constexpr int kMaxNbrBins = 512;

// Gaussian-gridding constants handed to the kernels by value.
struct GaussConst {
    double alpha;               // exponent scale: g(p) = exp(-alpha (p - delta)^2)
    double e3[2 * kMaxMsp];     // exp(-alpha p^2) for p = -msp+1 .. msp
};

}  // namespace nlf

// ---- the plan ------------------------------------------------------------------------------
struct nlf_plan {
    int dim, kernel, prec, batch, msp;
    int n[3], Mr[3];
    double L[3], h[3];
    double P, sigma;
    double eps = 0.0;           // confinement ratio (NLF_CONFINED2D)
    // split evaluation (3D Coulomb): I1 by this plan's FFTs, I2 by the ball plan `sub`
    int split = 0;
    double split_a = 0.0, split_P2 = 0.0;
    double* conv_e0 = nullptr;   // split: exp(-k0^2 / a) per axis-0 row of the padded grid (length Mr[0])
    int deterministic = 0;      // one work item per gather tile, plain stores; 3D plane-streamed interpolation
    int check_finite = 0;       // nlf_potential / nlf_type2 read the non-finite flag before returning
    int* nf_flag = nullptr;     // device: set to 1 by the density load pass on a NaN / Inf value
    nlf_plan* sub = nullptr;
    double pweight_a = 0.0;     // ball plan of a split: node weights times exp(-|k|^2 / a)
    int band = 0;               // ball plan of a split: spectrum cells |f_i| < band (3D) hold every
                                // value the interpolation reads and the spreading writes
    int n_r, n_theta, n_phi;
    long long N, G, M, Mh;      // grid points, oversampled grid points, nodes, half nodes
    hipStream_t stream;
    hipStream_t own_stream = nullptr;   // the solvers' graph-capturable stream (see solvers.hip)
    int tile[3];                // bin tile sizes per axis
    int window[3];              // tile + 2 msp - 1
    nlf::GaussConst gc;
    double st2;                 // prod h_i / Mr_i : raw interpolation sum -> rhohat
    double post;                // 1 / prod Mr_i   : inverse FFT normalisation

    // host copies (canonical order) for nlf_plan_nodes
    std::vector<double> k_host, w_host;

    // device buffers
    void* grid_a = nullptr;     // [batch][G] complex, type-2 grid
    void* grid_b = nullptr;     // [batch][G] complex, type-1 (spread) grid
    void* cbuf = nullptr;       // [batch][Mh] complex node values, sorted order
    double* s[3] = {nullptr, nullptr, nullptr};  // sorted node coordinates in oversampled cells
    double* wfac = nullptr;     // per sorted node: folded weight x symbol x constants
    double* gk = nullptr;       // per sorted node: exp(-sigma^2 |k|^2 / 2) (Laplace only)
    int* perm = nullptr;        // sorted node -> canonical half index
    nlf::Chunk* chunks = nullptr;
    int nchunks = 0;
    nlf::XcdSplit chunk_split{};   // chunks over the XCDs (2D interpolation)
    // output-driven spreading: per gather tile, the sorted nodes whose stencil overlaps it
    int gtile[3] = {1, 1, 1};
    int use_gather = 0;
    int* gcand = nullptr;
    nlf::GItem* gitems = nullptr;
    int ngitems = 0;
    nlf::XcdSplit item_split{};    // gather work items over the XCDs
    // deterministic plans: per-item partial sums of the tiles of several items, and those tiles
    double* pscratch = nullptr;    // [batch][nslots][256]
    long long pscratch_slots = 0;  // slots allocated
    long long nslots = 0;          // slots in use
    nlf::TileRed* tred = nullptr;
    long long tred_cap = 0;
    int ntred = 0;
    double* iacc = nullptr;     // [batch][Mh] complex FP64: tile-gathered interpolation sums
    void* wtab = nullptr;       // 2D gather plans: [Mh][8] (g, r) tile start weights (nufft.hip)
    void* itab = nullptr;       // 2D plans: [Mh][4][2] (g, r) interpolation start weights
    // spreading work decomposition (nlf_plan_set_spread / nlf_plan_autotune)
    int spread_mode = 0;        // NLF_SPREAD_GATHER or NLF_SPREAD_SCATTER
    int spread_kc = 64;         // candidates per block of the gather kernel
    int item_cap = nlf::kMItem; // candidates per work item
    std::vector<long long> gtile_off;   // explicit lists: per gather tile, first candidate
    int gng[3] = {1, 1, 1};     // gather tiles per axis
    long long gitems_cap = 0;   // GItem slots allocated on the device
    int items_bins = 0;         // the uploaded items index neighbour-bin streams
    // neighbour-bin gather (node bins = gather tiles)
    int gather_impl_ok = 0;
    int* bin_off = nullptr;     // [nbins + 1] first sorted node of each bin
    int impl_lo[3] = {0, 0, 0}, impl_n[3] = {1, 1, 1};   // neighbour bins per axis: t + lo .. t + lo + n - 1
    std::vector<long long> vtile_off;   // per tile: first candidate of its neighbour-bin stream
    double* dec[3] = {nullptr, nullptr, nullptr};   // 1 / c_g(j - n/2), length n_i
    void* tw_big[3] = {nullptr, nullptr, nullptr};  // twiddles of length Mr_i (plan precision)
    void* tw_small[3] = {nullptr, nullptr, nullptr};// twiddles of length n_i (solver FFTs)
    // type-1 side (spreading grid + inverse FFT) precision: the plan's, except FP32 3D plans with
    // output-driven spreading, which keep that side in FP64 (see plan.cpp)
    int t1_prec = 0;
    void* tw_t1[3] = {nullptr, nullptr, nullptr};
    double* mom = nullptr;      // [batch][4] moments m0, m1x, m1y (Laplace) ; scratch
    double* u11 = nullptr;      // Laplace only: u_{1,1}(x_j) on the grid [N], tabulated at plan time
    double* red = nullptr;      // reduction scratch
    size_t red_bytes = 0;
    long long workspace_bytes = 0;
    std::vector<void*> owned;   // every device allocation, freed on destroy

    // FP64 twin of an FP32 plan for the mixed gradient-flow schedule (created on first use)
    nlf_plan* twin = nullptr;
    nlf_box box_copy{};
    nlf_opts opts_copy{};

    // solver workspace (allocated by the first solver call; buffers are in `owned`)
    void* sws = nullptr;
    void (*sws_free)(void*) = nullptr;

    // stage timing
    int profiling = 0;
    std::vector<hipEvent_t> ev_pool;                 // created lazily, reused
    size_t ev_used = 0;
    std::vector<std::pair<int, std::pair<size_t, size_t>>> ev_marks;   // (stage, (start ev, stop ev))
    double stage_ms[NLF_NSTAGES] = {0};
    long long stage_cnt[NLF_NSTAGES] = {0};
};

namespace nlf {
int dev_alloc(nlf_plan* p, void** ptr, size_t bytes);
size_t elem_size(int prec);  // bytes of one complex element in the plan precision

// FFT front-ends (fft.hip)
int fft_type2_forward(nlf_plan* p, const void* rho);          // rho -> grid_a (pruned, fused precorrect)
int fft_type1_inverse(nlf_plan* p, void* u, bool add_u1);     // grid_b -> u (pruned, fused postcorrect)
int fft_split_i1(nlf_plan* p, const void* rho, void* u);      // u += I1 of a split (Eq. '3.9')
int fft_full(nlf_plan* p, void* data, int dir, int batch);    // n-grid complex FFT in place, all axes
int fill_zero(nlf_plan* p, void* ptr, size_t bytes);
int read_nonfinite(nlf_plan* p, int* seen);                   // sync the stream, read and clear nf_flag
int set_items(nlf_plan* p, int cap, bool bins);               // rebuild the gather work items

// NUFFT stages (nufft.hip)
// mode: 0 potential -> cbuf, 2 type-2 -> out; zero_b: the 2D kernel also clears grid_b
int interp(nlf_plan* p, int mode, void* out, bool zero_b);
int spread(nlf_plan* p);                                      // cbuf -> grid_b
int fold_c(nlf_plan* p, const void* c);                       // canonical full c -> cbuf (sorted, folded)
int potential(nlf_plan* p, const void* rho, void* u);
bool weight_table_fits(const nlf_plan* p);                    // 2D plans whose spreading can use a weight table
int build_weight_table(nlf_plan* p);                          // allocate and fill p->wtab (needs p->s)
int build_interp_table(nlf_plan* p);                          // 2D: allocate and fill p->itab (needs p->s, chunks)

// harmonic-oscillator Gaussian initial guesses of the plan's fields (unnormalised), solvers.hip
int ho_guess(nlf_plan* p, const nlf_phys* phys, void* out);

// stage timing: returns an opaque mark index (or -1 when profiling is off)
int stage_begin(nlf_plan* p);
int stage_end(nlf_plan* p, int stage, int mark);
}  // namespace nlf
