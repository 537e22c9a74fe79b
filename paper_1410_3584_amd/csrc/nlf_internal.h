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
    int n_r, n_theta, n_phi;
    long long N, G, M, Mh;      // grid points, oversampled grid points, nodes, half nodes
    hipStream_t stream;
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
    double* dec[3] = {nullptr, nullptr, nullptr};   // 1 / c_g(j - n/2), length n_i
    void* tw_big[3] = {nullptr, nullptr, nullptr};  // twiddles of length Mr_i (plan precision)
    void* tw_small[3] = {nullptr, nullptr, nullptr};// twiddles of length n_i (solver FFTs)
    double* mom = nullptr;      // [batch][4] moments m0, m1x, m1y (Laplace) ; scratch
    double* red = nullptr;      // reduction scratch
    size_t red_bytes = 0;
    long long workspace_bytes = 0;
    std::vector<void*> owned;   // every device allocation, freed on destroy
};

namespace nlf {
int dev_alloc(nlf_plan* p, void** ptr, size_t bytes);
size_t elem_size(int prec);  // bytes of one complex element in the plan precision

// FFT front-ends (fft.hip)
int fft_type2_forward(nlf_plan* p, const void* rho);          // rho -> grid_a (pruned, fused precorrect)
int fft_type1_inverse(nlf_plan* p, void* u, bool add_u1);     // grid_b -> u (pruned, fused postcorrect)
int fft_full(nlf_plan* p, void* data, int dir, int batch);    // n-grid complex FFT in place, all axes
int fill_zero(nlf_plan* p, void* ptr, size_t bytes);

// NUFFT stages (nufft.hip)
int moments(nlf_plan* p, const void* rho);
int interp(nlf_plan* p, int mode, void* out);                 // mode: 0 potential -> cbuf, 1 type-2 -> out
int spread(nlf_plan* p);                                      // cbuf -> grid_b
int fold_c(nlf_plan* p, const void* c);                       // canonical full c -> cbuf (sorted, folded)
int potential(nlf_plan* p, const void* rho, void* u);
}  // namespace nlf
