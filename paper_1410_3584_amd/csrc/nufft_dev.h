// Device code of the NUFFT stages (kernel bodies and their launch wrappers); the host side is in
// nufft.hip.  Included by nufft.hip and by solvers.hip (the persistent executor).
#pragma once
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "exec.h"
#include "nlf_internal.h"

namespace nlf {

template <typename T> __device__ __forceinline__ V2<T> mk2(T x, T y);
template <> __device__ __forceinline__ float2 mk2<float>(float x, float y) { return make_float2(x, y); }
template <> __device__ __forceinline__ double2 mk2<double>(double x, double y) { return make_double2(x, y); }

typedef double d4_t __attribute__((ext_vector_type(4)));


// index modulo an oversampled grid extent (always a power of two)
__device__ __forceinline__ int wrap(int v, int M) { return v & (M - 1); }

// Workgroup barrier for LDS traffic only: this wave's LDS operations have completed, then
// s_barrier.  __syncthreads() also waits for every outstanding global load (its fence covers
// global memory), which would drain loads issued ahead of the barrier for later blocks.
__device__ __forceinline__ void lds_barrier() { __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Separable Gaussian weights for one axis: w[q] = exp(-alpha (q - msp + 1 - delta)^2), computed as
// exp(-alpha delta^2) * exp(2 alpha delta)^p * exp(-alpha p^2) (Greengard-Lee fast gridding).
template <typename T, int MSP>
__device__ __forceinline__ void gauss_weights(double s, const GaussConst& gc, T (&w)[2 * MSP], int& l0) {
    double f = floor(s);
    l0 = (int)f;
    double d = s - f;
    double e1 = exp(-gc.alpha * d * d);
    double e2 = exp(2.0 * gc.alpha * d);
    double e2i = 1.0 / e2;
    double pw = e1;
    w[MSP - 1] = (T)(pw * gc.e3[MSP - 1]);
#pragma unroll
    for (int q = MSP; q < 2 * MSP; ++q) {
        pw *= e2;
        w[q] = (T)(pw * gc.e3[q]);
    }
    pw = e1;
#pragma unroll
    for (int q = MSP - 2; q >= 0; --q) {
        pw *= e2i;
        w[q] = (T)(pw * gc.e3[q]);
    }
}

// weight of plane offset a (0..2msp-1) along axis 0, for the 3D plane-streamed kernels
__device__ __forceinline__ double gauss1(double d, int a, int msp, double alpha) {
    double x = (double)(a - msp + 1) - d;
    return exp(-alpha * x * x);
}

enum { MODE_COULOMB = 0, MODE_LAPLACE = 1, MODE_TYPE2 = 2 };

struct NodeArgs {
    int dim;
    int Mr[3], tile[3], W[3];
    const double* s[3];
    const Chunk* chunks;
    int nchunks;
    GaussConst gc;
    XcdSplit csplit;        // chunks over the XCDs (2D interpolation)
    XcdSplit isplit;        // gather work items over the XCDs (3D interpolation, spreading)
    // 2D plans with a weight table (nlf_plan::wtab): per sorted node m, wtab[8 m + (t0 mod 4)] and
    // wtab[8 m + 4 + (t1 mod 4)] hold tile_start() at the first cell of gather tile t0 along axis 0
    // and t1 along axis 1, for the (at most 4 consecutive) tiles its stencil overlaps: the tiles
    // whose explicit candidate lists hold the node
    const double2* wtab;
    // 2D plans (nlf_plan::itab): per sorted node m and lane quarter ka = 0..3 of the per-bin
    // interpolation, itab[2 (4 m + ka)] = (g, r) of its y-weights and itab[2 (4 m + ka) + 1] of
    // its x-weights: the start values of the weight recurrences of k_binterp2 (FP64 plans,
    // binterp2_starts) or k_binterp2_32 (FP32 plans, binterp2_32_starts)
    const double2* itab;
};

struct EpiArgs {
    int mode;
    void* out;              // MODE_COULOMB/LAPLACE: cbuf [batch][Mh] sorted; MODE_TYPE2: [batch][M] canonical
    long long ostride;
    const double* wfac;
    const double* gk;
    const double* mom;      // [batch][4]: m0, m1x, m1y
    double st2;             // raw sum -> rhohat
    double kscale[3];       // k_i = s_i * kscale_i
    const int* perm;
    int hphi, n_phi, n_theta;
};

// chunk index of this workgroup: hardware workgroup ids go round-robin over the 8 XCDs; give each
// XCD a contiguous range of chunks so that chunks of one bin and its neighbours share its L2
__device__ __forceinline__ int chunk_id(int nchunks) {
    int b = blockIdx.x;
    int per = (nchunks + 7) >> 3;
    return (b & 7) * per + (b >> 3);
}
// entry of a cost-balanced split taken by this workgroup, or -1 (its XCD's range is shorter)
__device__ __forceinline__ int split_id(const XcdSplit& xs, int bx) {
    const int x = bx & 7, id = xs.s[x] + (bx >> 3);
    return id < xs.s[x + 1] ? id : -1;
}
__device__ __forceinline__ int split_id(const XcdSplit& xs) { return split_id(xs, (int)blockIdx.x); }

template <typename T>
__device__ __forceinline__ void epilogue(const EpiArgs& e, int batch, int node, double fx, double fy,
                                         double s0, double s1) {
    if (e.mode == MODE_TYPE2) {
        double rx = e.st2 * fx, ry = e.st2 * fy;
        int hm = e.perm[node];
        int ab = hm / e.hphi, c = hm - ab * e.hphi;
        long long m = (long long)ab * e.n_phi + c;
        long long mp;
        if (e.n_theta == 1) {
            mp = m + e.hphi;
        } else {
            int a = ab / e.n_theta, bb = ab - a * e.n_theta;
            mp = ((long long)a * e.n_theta + (e.n_theta - 1 - bb)) * e.n_phi + c + e.hphi;
        }
        V2<T>* o = reinterpret_cast<V2<T>*>(e.out) + (long long)batch * e.ostride;
        o[m] = mk2<T>((T)rx, (T)ry);
        o[mp] = mk2<T>((T)rx, (T)(-ry));
        return;
    }
    const double w = e.wfac[node];
    double cx, cy;
    if (e.mode == MODE_COULOMB) {
        // c = 2 (2pi)^-d w_m rhohat_m, the Jacobian cancels the Coulomb symbol (Eq. 'ifft')
        cx = w * fx;
        cy = w * fy;
    } else {
        // c = 2 (2pi)^-2 w_m W(k_m),
        // W(k) = [rhohat(k) - (m0 - i k.m1) exp(-sigma^2 |k|^2 / 2)] / |k|   (Eq. 'phi2fourier')
        const double* mo = e.mom + 4 * batch;
        const double rx = e.st2 * fx, ry = e.st2 * fy;
        const double g = e.gk[node];
        const double km1 = s0 * e.kscale[0] * mo[1] + s1 * e.kscale[1] * mo[2];
        cx = w * (rx - g * mo[0]);
        cy = w * (ry + g * km1);
    }
    V2<T>* o = reinterpret_cast<V2<T>*>(e.out) + (long long)batch * e.ostride;
    o[node] = mk2<T>((T)cx, (T)cy);
}

// ---- interpolation ----------------------------------------------------------------------------
template <typename T, int MSP>
__global__ void __launch_bounds__(kChunk) k_interp3(const V2<T>* __restrict__ grid, long long gstride,
                                                    NodeArgs na, EpiArgs ea) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V2<T>* win = reinterpret_cast<V2<T>*>(smem_raw);
    const int cid = chunk_id(na.nchunks);
    if (cid >= na.nchunks) return;
    const Chunk ch = na.chunks[cid];
    const int b = blockIdx.y;
    const V2<T>* g = grid + (long long)b * gstride;
    const int W1 = na.W[1], W2 = na.W[2];
    const int NP = na.tile[0] + 2 * MSP - 1;
    const int o0 = ch.t0 * na.tile[0] - MSP + 1;
    const int o1 = ch.t1 * na.tile[1] - MSP + 1, o2 = ch.t2 * na.tile[2] - MSP + 1;
    const long long plane = (long long)na.Mr[1] * na.Mr[2];
    const int t = threadIdx.x;
    const bool active = t < ch.count;
    const int node = ch.start + (active ? t : 0);
    T w1[2 * MSP], w2[2 * MSP];
    int l0 = 0, l1 = 0, l2 = 0;
    double d0 = 0;
    double sv0 = 0, sv1 = 0, sv2 = 0;
    int r0 = 0, r1 = 0, r2 = 0;
    if (active) {
        sv0 = na.s[0][node];
        sv1 = na.s[1][node];
        sv2 = na.s[2][node];
        double f0 = floor(sv0);
        l0 = (int)f0;
        d0 = sv0 - f0;
        gauss_weights<T, MSP>(sv1, na.gc, w1, l1);
        gauss_weights<T, MSP>(sv2, na.gc, w2, l2);
        r0 = wrap(l0, na.Mr[0]) - ch.t0 * na.tile[0];
        r1 = wrap(l1, na.Mr[1]) - ch.t1 * na.tile[1];
        r2 = wrap(l2, na.Mr[2]) - ch.t2 * na.tile[2];
    }
    double ax = 0, ay = 0;
    // a plane's window: every load of a thread is issued before its first LDS store
    constexpr int PER = ((8 + 2 * MSP - 1) * (8 + 2 * MSP - 1) + kChunk - 1) / kChunk;
    for (int q = 0; q < NP; ++q) {
        const V2<T>* gp = g + (long long)wrap(o0 + q, na.Mr[0]) * plane;
        V2<T> pv[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int idx = threadIdx.x + u * kChunk;
            if (idx < W1 * W2) {
                const int r = idx / W2, c = idx - r * W2;
                pv[u] = gp[(long long)wrap(o1 + r, na.Mr[1]) * na.Mr[2] + wrap(o2 + c, na.Mr[2])];
            }
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int idx = threadIdx.x + u * kChunk;
            if (idx < W1 * W2) win[idx] = pv[u];
        }
        __syncthreads();
        const int a = q - r0;
        if (active && a >= 0 && a < 2 * MSP) {
            double px = 0, py = 0;
            const V2<T>* base = win + r1 * W2 + r2;
#pragma unroll
            for (int i = 0; i < 2 * MSP; ++i) {
                T rx = 0, ry = 0;
                const V2<T>* row = base + i * W2;
#pragma unroll
                for (int j = 0; j < 2 * MSP; ++j) {
                    V2<T> v = row[j];
                    rx += v.x * w2[j];
                    ry += v.y * w2[j];
                }
                px += (double)w1[i] * (double)rx;
                py += (double)w1[i] * (double)ry;
            }
            double g0 = gauss1(d0, a, MSP, na.gc.alpha);
            ax += g0 * px;
            ay += g0 * py;
        }
        __syncthreads();
    }
    if (active) epilogue<T>(ea, b, node, ax, ay, sv0, sv1);
}

// ---- spreading ------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void lds_add(T* p, T v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ void global_add(T* p, T v) {
    unsafeAtomicAdd(p, v);
}

template <typename T, int MSP>
__global__ void __launch_bounds__(kChunk) k_spread2(V2<T>* __restrict__ grid, long long gstride,
                                                    const V2<T>* __restrict__ cbuf, long long cstride,
                                                    NodeArgs na) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V2<T>* win = reinterpret_cast<V2<T>*>(smem_raw);
    const int cid = chunk_id(na.nchunks);
    if (cid >= na.nchunks) return;
    const Chunk ch = na.chunks[cid];
    const int b = blockIdx.y;
    V2<T>* g = grid + (long long)b * gstride;
    const int W0 = na.W[0], W1 = na.W[1];
    const int o0 = ch.t0 * na.tile[0] - MSP + 1, o1 = ch.t1 * na.tile[1] - MSP + 1;
    for (int idx = threadIdx.x; idx < W0 * W1; idx += kChunk) win[idx] = mk2<T>(0, 0);
    __syncthreads();
    const int t = threadIdx.x;
    if (t < ch.count) {
        const int node = ch.start + t;
        T w0[2 * MSP], w1[2 * MSP];
        int l0, l1;
        gauss_weights<T, MSP>(na.s[0][node], na.gc, w0, l0);
        gauss_weights<T, MSP>(na.s[1][node], na.gc, w1, l1);
        const int r0 = wrap(l0, na.Mr[0]) - ch.t0 * na.tile[0];
        const int r1 = wrap(l1, na.Mr[1]) - ch.t1 * na.tile[1];
        const V2<T> c = cbuf[(long long)b * cstride + node];
        V2<T>* base = win + r0 * W1 + r1;
#pragma unroll
        for (int i = 0; i < 2 * MSP; ++i) {
            const T cx = c.x * w0[i], cy = c.y * w0[i];
            T* row = reinterpret_cast<T*>(base + i * W1);
#pragma unroll
            for (int j = 0; j < 2 * MSP; ++j) {
                lds_add<T>(row + 2 * j, cx * w1[j]);
                lds_add<T>(row + 2 * j + 1, cy * w1[j]);
            }
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < W0 * W1; idx += kChunk) {
        int r = idx / W1, c = idx - r * W1;
        V2<T> v = win[idx];
        if (v.x != (T)0 || v.y != (T)0) {
            T* dst = reinterpret_cast<T*>(g + (long long)wrap(o0 + r, na.Mr[0]) * na.Mr[1] + wrap(o1 + c, na.Mr[1]));
            global_add<T>(dst, v.x);
            global_add<T>(dst + 1, v.y);
        }
    }
}

template <typename T, int MSP>
__global__ void __launch_bounds__(kChunk) k_spread3(V2<T>* __restrict__ grid, long long gstride,
                                                    const V2<T>* __restrict__ cbuf, long long cstride,
                                                    NodeArgs na) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V2<T>* win = reinterpret_cast<V2<T>*>(smem_raw);
    const int cid = chunk_id(na.nchunks);
    if (cid >= na.nchunks) return;
    const Chunk ch = na.chunks[cid];
    const int b = blockIdx.y;
    V2<T>* g = grid + (long long)b * gstride;
    const int W1 = na.W[1], W2 = na.W[2];
    const int NP = na.tile[0] + 2 * MSP - 1;
    const int o0 = ch.t0 * na.tile[0] - MSP + 1;
    const int o1 = ch.t1 * na.tile[1] - MSP + 1, o2 = ch.t2 * na.tile[2] - MSP + 1;
    const long long plane = (long long)na.Mr[1] * na.Mr[2];
    const int t = threadIdx.x;
    const bool active = t < ch.count;
    const int node = ch.start + (active ? t : 0);
    T w1[2 * MSP], w2[2 * MSP];
    int l0 = 0, l1 = 0, l2 = 0;
    double d0 = 0;
    int r0 = 0, r1 = 0, r2 = 0;
    V2<T> c = mk2<T>(0, 0);
    if (active) {
        double sv0 = na.s[0][node];
        double f0 = floor(sv0);
        l0 = (int)f0;
        d0 = sv0 - f0;
        gauss_weights<T, MSP>(na.s[1][node], na.gc, w1, l1);
        gauss_weights<T, MSP>(na.s[2][node], na.gc, w2, l2);
        r0 = wrap(l0, na.Mr[0]) - ch.t0 * na.tile[0];
        r1 = wrap(l1, na.Mr[1]) - ch.t1 * na.tile[1];
        r2 = wrap(l2, na.Mr[2]) - ch.t2 * na.tile[2];
        c = cbuf[(long long)b * cstride + node];
    }
    for (int idx = threadIdx.x; idx < W1 * W2; idx += kChunk) win[idx] = mk2<T>(0, 0);
    __syncthreads();
    for (int q = 0; q < NP; ++q) {
        const int a = q - r0;
        if (active && a >= 0 && a < 2 * MSP) {
            const T g0 = (T)gauss1(d0, a, MSP, na.gc.alpha);
            V2<T>* base = win + r1 * W2 + r2;
#pragma unroll
            for (int i = 0; i < 2 * MSP; ++i) {
                const T f = g0 * w1[i];
                const T cx = c.x * f, cy = c.y * f;
                T* row = reinterpret_cast<T*>(base + i * W2);
#pragma unroll
                for (int j = 0; j < 2 * MSP; ++j) {
                    lds_add<T>(row + 2 * j, cx * w2[j]);
                    lds_add<T>(row + 2 * j + 1, cy * w2[j]);
                }
            }
        }
        __syncthreads();
        V2<T>* gp = g + (long long)wrap(o0 + q, na.Mr[0]) * plane;
        for (int idx = threadIdx.x; idx < W1 * W2; idx += kChunk) {
            int r = idx / W2, cc = idx - r * W2;
            V2<T> v = win[idx];
            if (v.x != (T)0 || v.y != (T)0) {
                T* dst = reinterpret_cast<T*>(gp + (long long)wrap(o1 + r, na.Mr[1]) * na.Mr[2] + wrap(o2 + cc, na.Mr[2]));
                global_add<T>(dst, v.x);
                global_add<T>(dst + 1, v.y);
                win[idx] = mk2<T>(0, 0);
            }
        }
        __syncthreads();
    }
}

// ---- output-driven spreading (gather over candidate nodes, no LDS atomics) ----------------------
// Weights of one node along one axis on the GT cells o..o+GT-1 of a gather tile.
// When Mr >= 2 msp + GT every cell has one offset p = (cell - l0) mod Mr near the stencil, and the
// weight is exp(-alpha (p - delta)^2), stepped by its ratio exp(-alpha (2 (p - delta) + 1)), itself
// stepped by exp(-2 alpha) (two exps per axis, two multiplies per cell).  Cells of the tile outside
// the node's 2 msp stencil keep their Gaussian weight instead of 0: it is below e^{-3 pi msp / 4},
// the truncation level of the stencil itself.  Otherwise (small grids, where the stencil wraps onto
// itself) the weight is the sum over the stencil offsets p == cell - l0 (mod Mr), p in [-msp+1, msp].
// (g, r) of a node at cell o when Mr >= 2 msp + GT: the weight g = exp(-alpha x^2) at the cell's
// offset x from the node and the ratio r = exp(-alpha (2 x + 1)) to the next cell.  The offset is
// the representative in (msp - Mr, msp], which holds every offset a tile overlapping the stencil
// can have (-msp - GT + 2 .. msp).
__device__ __forceinline__ double2 tile_start(double s, int o, int Mr, int msp, double alpha) {
    const double f = floor(s);
    const int l0 = (int)f;
    const double d = s - f;
    int p0 = wrap(o - l0 + msp - 1, Mr) - msp + 1;
    if (p0 > msp) p0 -= Mr;
    const double x = (double)p0 - d;
    return make_double2(exp(-alpha * x * x), exp(-alpha * (2.0 * x + 1.0)));
}

template <int MSP, int GT>
__device__ __forceinline__ void tile_weights(double s, int o, int Mr, double alpha, double qq, double (&w)[GT]) {
    if (Mr >= 2 * MSP + GT) {
        const double2 gr = tile_start(s, o, Mr, MSP, alpha);
        double g = gr.x, r = gr.y;
#pragma unroll
        for (int k = 0; k < GT; ++k) {
            w[k] = g;
            g *= r;
            r *= qq;
        }
    } else {
        const double f = floor(s);
        const int l0 = (int)f;
        const double d = s - f;
#pragma unroll
        for (int k = 0; k < GT; ++k) {
            double acc = 0;
            for (int pp = wrap(o + k - l0 + MSP - 1, Mr) - MSP + 1; pp <= MSP; pp += Mr) {
                double x = (double)pp - d;
                acc += exp(-alpha * x * x);
            }
            w[k] = acc;
        }
    }
}

// The sum a gather tile receives from a block of K candidate nodes,
//   F[x][y] = sum_k c_k w0_k[x] w1_k[y]            (2D tile: 8 x 16 cells)
//   F[x][(y,z)] = sum_k c_k w0_k[x] w1_k[y] w2_k[z]  (3D tile: 8 x 4 x 4 cells),
// is the product A^T B of the K x 16 matrices A[k][(comp, x)] = (Re|Im c_k) w0_k[x] and
// B[k][j] = w1_k[y] (2D) or w1_k[y] w2_k[z] (3D, j = 4y + z): a dense contraction over the
// candidates, run on the FP64 matrix cores, 4 candidates per v_mfma_f64_16x16x4.
//
// Phase 1: thread t < K builds row t of A, thread K + t row t of B (rows past the item's count are
// zero), in LDS rows of 16 doubles whose 16-byte chunks are XOR-swizzled by the row index so that
// the per-thread row stores hit distinct banks.  Phase 2: wave w multiplies candidates
// [w K/4, (w+1) K/4).  Phase 3: the four partial 16 x 16 tiles are summed through LDS and added
// to the grid with one FP64 (or FP32) atomic per cell component.
__device__ __forceinline__ int mrow_slot(int k, int chunk) {
    return ((chunk ^ ((k >> 1) & 7) ^ ((k & 1) << 2)) & 7);
}

// Neighbour-bin candidate streams: the node bins have the tile's shape; tile t reads the bins
// t + lo_i .. t + lo_i + n_i - 1 (periodic) in lexicographic order, each bin a contiguous range
// of sorted nodes.
struct BinArgs {
    const int* bin_off;     // [nbins + 1] first sorted node of each bin
    int lo[3], n[3], NB[3];
};

// The table of tile (g0, g1, g2)'s neighbour bins in LDS: pref[i] = candidates before bin i of the
// stream (pref[nbn] = total), start[i] = its first node.  Every thread of the workgroup calls it.
template <int NT>
__device__ __forceinline__ int bin_table(const BinArgs& ba, int g0, int g1, int g2, int* pref, int* tmp,
                                         int* start) {
    const int nbn = ba.n[0] * ba.n[1] * ba.n[2];
    const int t = threadIdx.x;
    for (int i = t; i < nbn; i += NT) {
        const int ia = i / (ba.n[1] * ba.n[2]), ib = (i / ba.n[2]) % ba.n[1], ic = i % ba.n[2];
        const int b0 = (g0 + ba.lo[0] + ia + ba.NB[0]) % ba.NB[0];
        const int b1 = (g1 + ba.lo[1] + ib + ba.NB[1]) % ba.NB[1];
        const int b2 = (g2 + ba.lo[2] + ic + ba.NB[2]) % ba.NB[2];
        const long long bid = ((long long)b0 * ba.NB[1] + b1) * ba.NB[2] + b2;
        const int s0 = ba.bin_off[bid];
        start[i] = s0;
        pref[i + 1] = ba.bin_off[bid + 1] - s0;
    }
    if (t == 0) pref[0] = 0;
    __syncthreads();
    // inclusive scan of pref[1..nbn] (Hillis-Steele, ping-pong through tmp)
    int* a = pref;
    int* c = tmp;
    for (int d = 1; d < nbn; d <<= 1) {
        for (int i = 1 + t; i <= nbn; i += NT) c[i] = a[i] + ((i - d >= 1) ? a[i - d] : 0);
        if (t == 0) c[0] = 0;
        __syncthreads();
        int* x = a;
        a = c;
        c = x;
    }
    if (a != pref) {
        for (int i = t; i <= nbn; i += NT) pref[i] = a[i];
        __syncthreads();
    }
    return nbn;
}

// sorted node at position pos (0 <= pos < pref[nbn]) of a neighbour-bin stream
__device__ __forceinline__ int bin_node(const int* pref, const int* start, int nbn, int pos) {
    int lo = 0, hi = nbn;   // pref[lo] <= pos < pref[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pref[mid] <= pos) lo = mid;
        else hi = mid;
    }
    return start[lo] + (pos - pref[lo]);
}

template <bool BINS>
__host__ __device__ constexpr int bin_table_lds() {
    return BINS ? (2 * (kMaxNbrBins + 1) + kMaxNbrBins) * (int)sizeof(int) : 0;
}
template <int KC, bool BINS>
__host__ __device__ constexpr int mspread_lds() {
    return 2 * KC * 16 * (int)sizeof(double) + bin_table_lds<BINS>();
}

template <typename T, typename TG, int MSP, int DIM, int KC, bool BINS, bool WT = false>
__device__ __forceinline__ void mspread_body(V2<TG>* __restrict__ grid, long long gstride,
                                             const V2<T>* __restrict__ cbuf, long long cstride,
                                             const NodeArgs& na, const GItem* __restrict__ items, int nitems,
                                             const int* __restrict__ cand, double qq, const BinArgs& ba,
                                             double* __restrict__ pscr, long long sstride, VBlk vb,
                                             unsigned char* smem) {
    static_assert(!WT || DIM == 2, "weight tables are 2D");
    constexpr int NW = 2 * KC / 64;   // waves; each multiplies KC / NW candidates of a block
    static_assert(KC % (4 * NW) == 0 && (KC / NW) % 8 == 0, "whole pairs of MFMA steps per wave");
    static_assert(2 * KC * 16 >= NW * 4 * 64, "wave partials fit S");
    double* S = reinterpret_cast<double*>(smem);
    const int iid = split_id(na.isplit, vb.x);
    if (iid < 0) return;
    const GItem it = items[iid];
    const int b = vb.y;
    const int t = threadIdx.x;
    const int o0 = it.g0 * 8;
    const int o1 = it.g1 * (DIM == 2 ? 16 : 4);
    const int o2 = it.g2 * 4;
    const int k = t & (KC - 1);
    const bool is_a = t < KC;
    const int wv = t >> 6, lane = t & 63;
    const int r = lane & 15;
    const int kb = wv * (KC / NW);
    // the weight-table slot of this thread's axis (A rows: axis 0, B rows: axis 1)
    const int wslot = is_a ? (it.g0 & 3) : 4 + (it.g1 & 3);
    // four accumulators: independent product chains keep the FP64 matrix pipe busy
    d4_t acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0, acc2 = acc0, acc3 = acc0;
    // neighbour-bin streams: the tile's bin table (pref, start) in LDS
    int* nb_pref = reinterpret_cast<int*>(smem + 2 * KC * 16 * sizeof(double));
    int* nb_tmp = nb_pref + (kMaxNbrBins + 1);
    int* nb_start = nb_tmp + (kMaxNbrBins + 1);
    int nbn = 0;
    if (BINS) nbn = bin_table<2 * KC>(ba, it.g0, it.g1, it.g2, nb_pref, nb_tmp, nb_start);
    // Node data of this thread's candidate, loaded one block ahead so that the loads overlap the
    // previous block's matrix products.
    auto node_at = [&](int base) -> int {
        if (WT) return cand[it.start + min(base + k, it.count - 1)];   // unconditional: see fetch
        if (base + k >= it.count) return -1;
        return BINS ? bin_node(nb_pref, nb_start, nbn, (int)it.start + base + k) : cand[it.start + base + k];
    };
    struct NodeData {
        double sa, sb;
        double2 wgr;   // WT: (g, r) of the candidate on this thread's tile axis
        double m;      // WT: 1, or 0 past the item's count (zero rows)
        V2<T> cv;
    };
    // WT: every lane loads, whether or not its candidate exists (past the count the last one
    // stands in, multiplied by m = 0), and the B lanes load the node value too: unconditional
    // loads, which the compiler's wait counts track exactly
    auto fetch = [&](NodeData& d, int node, int base) {
        if (WT) {
            d.wgr = na.wtab[8 * (long long)node + wslot];
            d.cv = cbuf[(long long)b * cstride + node];
            d.m = (base + k < it.count) ? 1.0 : 0.0;
            return;
        }
        if (node >= 0) {
            if (is_a) {
                if (!WT) d.sa = na.s[0][node];
                d.cv = cbuf[(long long)b * cstride + node];
            } else if (!WT) {
                d.sa = na.s[1][node];
                if (DIM == 3) d.sb = na.s[2][node];
            }
        }
    };
    NodeData d0{};
    fetch(d0, node_at(0), 0);
    // the candidate index runs one block ahead of the node data it addresses, so that the data's
    // loads do not wait for the index load's latency
    int nxt = node_at(KC);
    auto block = [&](int base, NodeData& d) {
        const int cnt = min(KC, it.count - base);
        if (base > 0) lds_barrier();   // the previous block's products have read S
        double row[16];
        if (WT) {   // absent candidates have m = 0 (see fetch): no branch, no zeroing
            double g = d.wgr.x * d.m, rr = d.wgr.y;
            if (is_a) {
                double gx = (double)d.cv.x * g, gy = (double)d.cv.y * g;
#pragma unroll
                for (int x = 0; x < 8; ++x) {
                    row[x] = gx;
                    row[8 + x] = gy;
                    gx *= rr;
                    gy *= rr;
                    rr *= qq;
                }
            } else {
#pragma unroll
                for (int y = 0; y < 16; ++y) {
                    row[y] = g;
                    g *= rr;
                    rr *= qq;
                }
            }
        } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) row[j] = 0.0;
        if (k < cnt) {
            if (is_a) {
                double w0[8];
                tile_weights<MSP, 8>(d.sa, o0, na.Mr[0], na.gc.alpha, qq, w0);
                const double cx = (double)d.cv.x, cy = (double)d.cv.y;
#pragma unroll
                for (int x = 0; x < 8; ++x) {
                    row[x] = cx * w0[x];
                    row[8 + x] = cy * w0[x];
                }
            } else if (DIM == 2) {
                tile_weights<MSP, 16>(d.sa, o1, na.Mr[1], na.gc.alpha, qq, row);
            } else {
                double w1[4], w2[4];
                tile_weights<MSP, 4>(d.sa, o1, na.Mr[1], na.gc.alpha, qq, w1);
                tile_weights<MSP, 4>(d.sb, o2, na.Mr[2], na.gc.alpha, qq, w2);
#pragma unroll
                for (int y = 0; y < 4; ++y)
#pragma unroll
                    for (int z = 0; z < 4; ++z) row[4 * y + z] = w1[y] * w2[z];
            }
        }
        }
        double* mine = S + (is_a ? 0 : KC * 16) + k * 16;
#pragma unroll
        for (int c = 0; c < 8; ++c)
            *reinterpret_cast<double2*>(mine + 2 * mrow_slot(k, c)) = make_double2(row[2 * c], row[2 * c + 1]);
        lds_barrier();
        fetch(d, nxt, base + KC);   // the next block's (this block's weights are built)
        nxt = node_at(base + 2 * KC);
        if (kb < cnt) {   // rows past the count are zero: whole steps, fully unrolled
            constexpr int kSteps = KC / NW / 4;
            double av[kSteps], bv[kSteps];
#pragma unroll
            for (int q = 0; q < kSteps; ++q) {
                const int kk = kb + 4 * q + (lane >> 4);
                const int off = kk * 16 + 2 * mrow_slot(kk, r >> 1) + (r & 1);
                av[q] = S[off];
                bv[q] = S[KC * 16 + off];
            }
            static_assert(kSteps % 4 == 0, "four chains");
            if constexpr (WT) {
                // one product chain: the FP64 matrix pipe issues at the same rate with one chain as
                // with four, and the 24 registers saved admit a fifth wave per SIMD
#pragma unroll
                for (int q = 0; q < kSteps; ++q) acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc0, 0, 0, 0);
            } else {
#pragma unroll
                for (int q = 0; q < kSteps; q += 4) {
                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q + 1], bv[q + 1], acc1, 0, 0, 0);
                    acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q + 2], bv[q + 2], acc2, 0, 0, 0);
                    acc3 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q + 3], bv[q + 3], acc3, 0, 0, 0);
                }
            }
        }
    };
    for (int base = 0; base < it.count; base += KC) block(base, d0);
    const d4_t acc = (acc0 + acc1) + (acc2 + acc3);
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) S[(wv * 4 + v) * 64 + lane] = acc[v];
    __syncthreads();
    // v_mfma_f64_16x16x4 leaves element (i, j) of the 16 x 16 product in register v = i / 4 of
    // lane l = 16 (i mod 4) + j
    for (int o = t; o < 256; o += 2 * KC) {
        const int v = o >> 6, l = o & 63;
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) sum += S[(w * 4 + v) * 64 + l];
        const int i = 4 * v + (l >> 4), j = l & 15;
        if (pscr && !it.only) {   // deterministic plan: the item's partial sum, every cell
            pscr[(long long)b * sstride + (long long)it.slot * 256 + o] = sum;
            continue;
        }
        if (it.only || sum != 0.0) {
            const int x = o0 + (i & 7);
            long long cell;
            if (DIM == 2)
                cell = (long long)x * na.Mr[1] + o1 + j;
            else
                cell = ((long long)x * na.Mr[1] + o1 + (j >> 2)) * na.Mr[2] + o2 + (j & 3);
            TG* dst = reinterpret_cast<TG*>(grid + (long long)b * gstride + cell) + (i >> 3);
            // the tile's only item owns its cells: a plain store; otherwise one atomic per item
            if (it.only) *dst = (TG)sum;
            else global_add<TG>(dst, (TG)sum);
        }
    }
}

// (weight-table plans: 5 waves per SIMD, all that 16 KiB of LDS per workgroup admits, with one
// product chain; the other variants keep 4)
template <typename T, typename TG, int MSP, int DIM, int KC, bool BINS, bool WT>
__global__ void __launch_bounds__(2 * KC, (WT && mspread_lds<KC, BINS>() <= 16384) ? 5 : 4) k_mspread(V2<TG>* __restrict__ grid, long long gstride,
                                                        const V2<T>* __restrict__ cbuf, long long cstride,
                                                        NodeArgs na, const GItem* __restrict__ items, int nitems,
                                                        const int* __restrict__ cand, double qq, BinArgs ba,
                                                        double* __restrict__ pscr, long long sstride) {
    __shared__ __align__(16) unsigned char smem[mspread_lds<KC, BINS>()];
    mspread_body<T, TG, MSP, DIM, KC, BINS, WT>(grid, gstride, cbuf, cstride, na, items, nitems, cand, qq, ba, pscr,
                                                sstride, hw_block(), smem);
}

// The same gather on the FP32 matrix cores, for FP32 plans (v_mfma_f32_16x16x4f32, twice the FP64
// matrix rate).  The rows of A and B are built as in k_mspread (weights in FP64, rounded to FP32)
// and kept transposed in LDS, SA[j][k] / SB[j][k] with a pitch of KC + 4 floats: the per-thread
// stores of one row hit consecutive banks, and the MFMA operand reads (16 rows j, 4 candidates k)
// are conflict-free within each half-wave.  Each block of KC candidates is summed in FP32 (the
// wave's K/NW candidates over four product chains); the blocks are added in FP64, and the item's
// sum goes to the FP64 spreading grid of the FP32 plan.
typedef float f4_t __attribute__((ext_vector_type(4)));

// row of the 16 x 16 result held by accumulator register v of lane l (column l mod 16) of
// v_mfma_f32_16x16x4f32
__device__ __forceinline__ int mfma32_row(int v, int l) { return 4 * (l >> 4) + v; }

template <int KC, bool BINS>
__host__ __device__ constexpr int mspread32_lds() {
    return 2 * 16 * (KC + 4) * (int)sizeof(float) + (2 * KC / 64) * 4 * 64 * (int)sizeof(double) +
           bin_table_lds<BINS>();
}

template <int MSP, int DIM, int KC, bool BINS, bool WT = false>
__device__ __forceinline__ void mspread32_body(double2* __restrict__ grid, long long gstride,
                                               const float2* __restrict__ cbuf, long long cstride,
                                               const NodeArgs& na, const GItem* __restrict__ items, int nitems,
                                               const int* __restrict__ cand, double qq, const BinArgs& ba,
                                               double* __restrict__ pscr, long long sstride, VBlk vb,
                                               unsigned char* smem) {
    static_assert(!WT || DIM == 2, "weight tables are 2D");
    constexpr int NW = 2 * KC / 64;
    constexpr int KP = KC + 4;
    static_assert((KC / NW) % 16 == 0, "whole groups of four MFMA steps per wave");
    double* R = reinterpret_cast<double*>(smem);
    float* SA = reinterpret_cast<float*>(smem + NW * 4 * 64 * sizeof(double));
    float* SB = SA + 16 * KP;
    const int iid = split_id(na.isplit, vb.x);
    if (iid < 0) return;
    const GItem it = items[iid];
    const int b = vb.y;
    const int t = threadIdx.x;
    const int o0 = it.g0 * 8;
    const int o1 = it.g1 * (DIM == 2 ? 16 : 4);
    const int o2 = it.g2 * 4;
    const int k = t & (KC - 1);
    const bool is_a = t < KC;
    const int wv = t >> 6, lane = t & 63;
    const int r = lane & 15, kq = lane >> 4;
    const int kb = wv * (KC / NW);
    const int wslot = is_a ? (it.g0 & 3) : 4 + (it.g1 & 3);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int* nb_pref = reinterpret_cast<int*>(SB + 16 * KP);
    int* nb_tmp = nb_pref + (kMaxNbrBins + 1);
    int* nb_start = nb_tmp + (kMaxNbrBins + 1);
    int nbn = 0;
    if (BINS) nbn = bin_table<2 * KC>(ba, it.g0, it.g1, it.g2, nb_pref, nb_tmp, nb_start);
    // node data one block ahead, as in mspread_body
    auto node_at = [&](int base) -> int {
        if (WT) return cand[it.start + min(base + k, it.count - 1)];   // unconditional: see fetch
        if (base + k >= it.count) return -1;
        return BINS ? bin_node(nb_pref, nb_start, nbn, (int)it.start + base + k) : cand[it.start + base + k];
    };
    struct NodeData {
        double sa, sb;
        double2 wgr;
        double m;
        float2 cv;
    };
    auto fetch = [&](NodeData& d, int node, int base) {   // as in mspread_body
        if (WT) {
            d.wgr = na.wtab[8 * (long long)node + wslot];
            d.cv = cbuf[(long long)b * cstride + node];
            d.m = (base + k < it.count) ? 1.0 : 0.0;
            return;
        }
        if (node >= 0) {
            if (is_a) {
                if (!WT) d.sa = na.s[0][node];
                d.cv = cbuf[(long long)b * cstride + node];
            } else if (!WT) {
                d.sa = na.s[1][node];
                if (DIM == 3) d.sb = na.s[2][node];
            }
        }
    };
    NodeData d0{};
    fetch(d0, node_at(0), 0);
    int nxt = node_at(KC);   // the candidate index one block ahead of its data, as in mspread_body
    auto block = [&](int base, NodeData& d) {
        const int cnt = min(KC, it.count - base);
        if (base > 0) lds_barrier();   // the previous block's products have read SA, SB
        float row[16];
        if (WT) {   // absent candidates have m = 0 (see fetch): no branch, no zeroing
            double g = d.wgr.x * d.m, rr = d.wgr.y;
            if (is_a) {
                double gx = (double)d.cv.x * g, gy = (double)d.cv.y * g;
#pragma unroll
                for (int x = 0; x < 8; ++x) {
                    row[x] = (float)gx;
                    row[8 + x] = (float)gy;
                    gx *= rr;
                    gy *= rr;
                    rr *= qq;
                }
            } else {
#pragma unroll
                for (int y = 0; y < 16; ++y) {
                    row[y] = (float)g;
                    g *= rr;
                    rr *= qq;
                }
            }
        } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) row[j] = 0.0f;
        if (k < cnt) {
            if (is_a) {
                double w0[8];
                tile_weights<MSP, 8>(d.sa, o0, na.Mr[0], na.gc.alpha, qq, w0);
                const double cx = (double)d.cv.x, cy = (double)d.cv.y;
#pragma unroll
                for (int x = 0; x < 8; ++x) {
                    row[x] = (float)(cx * w0[x]);
                    row[8 + x] = (float)(cy * w0[x]);
                }
            } else if (DIM == 2) {
                double w1[16];
                tile_weights<MSP, 16>(d.sa, o1, na.Mr[1], na.gc.alpha, qq, w1);
#pragma unroll
                for (int j = 0; j < 16; ++j) row[j] = (float)w1[j];
            } else {
                double w1[4], w2[4];
                tile_weights<MSP, 4>(d.sa, o1, na.Mr[1], na.gc.alpha, qq, w1);
                tile_weights<MSP, 4>(d.sb, o2, na.Mr[2], na.gc.alpha, qq, w2);
#pragma unroll
                for (int y = 0; y < 4; ++y)
#pragma unroll
                    for (int z = 0; z < 4; ++z) row[4 * y + z] = (float)(w1[y] * w2[z]);
            }
        }
        }
        float* dst = is_a ? SA : SB;
#pragma unroll
        for (int j = 0; j < 16; ++j) dst[j * KP + k] = row[j];
        lds_barrier();
        fetch(d, nxt, base + KC);   // the next block's (this block's weights are built)
        nxt = node_at(base + 2 * KC);
        if (kb < cnt) {   // rows past the count are zero: whole steps, fully unrolled
            constexpr int kSteps = KC / NW / 4;
            f4_t c0 = {0.0f, 0.0f, 0.0f, 0.0f}, c1 = c0, c2 = c0, c3 = c0;
#pragma unroll
            for (int q = 0; q < kSteps; q += 4) {
                const int off = r * KP + kb + 4 * q + kq;
                c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(SA[off], SB[off], c0, 0, 0, 0);
                c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(SA[off + 4], SB[off + 4], c1, 0, 0, 0);
                c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(SA[off + 8], SB[off + 8], c2, 0, 0, 0);
                c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(SA[off + 12], SB[off + 12], c3, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] += (double)((c0[v] + c1[v]) + (c2[v] + c3[v]));
        }
    };
    for (int base = 0; base < it.count; base += KC) block(base, d0);
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) R[(wv * 4 + v) * 64 + lane] = acc[v];
    __syncthreads();
    for (int o = t; o < 256; o += 2 * KC) {
        const int v = o >> 6, l = o & 63;
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) sum += R[(w * 4 + v) * 64 + l];
        const int i = mfma32_row(v, l), j = l & 15;
        if (pscr && !it.only) {   // deterministic plan: the item's partial sum, every cell, in the
                                  // slot order k_tile_reduce reads (the FP64 product's layout)
            pscr[(long long)b * sstride + (long long)it.slot * 256 + 64 * (i >> 2) + 16 * (i & 3) + j] = sum;
            continue;
        }
        if (it.only || sum != 0.0) {
            const int x = o0 + (i & 7);
            long long cell;
            if (DIM == 2)
                cell = (long long)x * na.Mr[1] + o1 + j;
            else
                cell = ((long long)x * na.Mr[1] + o1 + (j >> 2)) * na.Mr[2] + o2 + (j & 3);
            double* d = reinterpret_cast<double*>(grid + (long long)b * gstride + cell) + (i >> 3);
            if (it.only) *d = sum;
            else global_add<double>(d, sum);
        }
    }
}

template <int MSP, int DIM, int KC, bool BINS, bool WT>
__global__ void __launch_bounds__(2 * KC, 4) k_mspread32(double2* __restrict__ grid, long long gstride,
                                                          const float2* __restrict__ cbuf, long long cstride,
                                                          NodeArgs na, const GItem* __restrict__ items, int nitems,
                                                          const int* __restrict__ cand, double qq, BinArgs ba,
                                                          double* __restrict__ pscr, long long sstride) {
    __shared__ __align__(16) unsigned char smem[mspread32_lds<KC, BINS>()];
    mspread32_body<MSP, DIM, KC, BINS, WT>(grid, gstride, cbuf, cstride, na, items, nitems, cand, qq, ba, pscr, sstride,
                                           hw_block(), smem);
}

// Deterministic plans: a tile of several work items adds its items' partial sums in slot order
// and stores the result (cell o of the tile as in k_mspread's write-back), so no atomics decide the
// order of the additions.
template <typename TG, int DIM>
__global__ void __launch_bounds__(256) k_tile_reduce(V2<TG>* __restrict__ grid, long long gstride,
                                                     const double* __restrict__ pscr, long long sstride,
                                                     const TileRed* __restrict__ tr, NodeArgs na) {
    const TileRed r = tr[blockIdx.x];
    const int b = blockIdx.y;
    const int o = threadIdx.x;
    const double* src = pscr + (long long)b * sstride + (long long)r.first * 256 + o;
    double sum = 0.0;
    for (int s = 0; s < r.n; ++s) sum += src[(long long)s * 256];
    const int v = o >> 6, l = o & 63;
    const int i = 4 * v + (l >> 4), j = l & 15;
    const int x = r.g0 * 8 + (i & 7);
    long long cell;
    if (DIM == 2)
        cell = (long long)x * na.Mr[1] + r.g1 * 16 + j;
    else
        cell = ((long long)x * na.Mr[1] + r.g1 * 4 + (j >> 2)) * na.Mr[2] + r.g2 * 4 + (j & 3);
    TG* dst = reinterpret_cast<TG*>(grid + (long long)b * gstride + cell) + (i >> 3);
    *dst = (TG)sum;
}

// ---- 2D interpolation on the FP64 matrix cores, one workgroup per bin of nodes -----------------
// The nodes of one chunk have l0 in the same 8 x 16 bin, so their stencils lie in one window of
// (8 + 2 msp - 1) x (16 + 2 msp - 1) cells, staged in LDS as FP64 real and imaginary planes.  For
// a group of 16 nodes and an 8-row block of the window,
//   H[(comp, x)][k] = sum_y G_comp[x][y] w1_k[y]
// is a 16 x 16 x (4 KS) product (KS v_mfma_f64_16x16x4 steps; A = window values, B = the nodes'
// y-weights, zero outside each stencil), and u_k = sum_x w0_k[x] H[x][k] accumulates in registers
// over the row blocks.  Wave w owns groups w, w + 4: lane (ia, ka) = (l mod 16, l / 16) holds node
// 16 g + ia, its y-weights on columns 4 st + ka and its x-weights on rows 4 m + ka, both from the
// Gaussian recurrence g(x + 4) = g(x) exp(-alpha (8 x + 16)), whose ratio steps by exp(-32 alpha)
// (four exps per lane and group).  The plan orders each bin's nodes by column offset, so a group
// multiplies only the k-steps its nodes' stencils touch.  The node's complex sum goes through the
// FP64 epilogue (symbol times weight) directly: no atomics, no cross-wave reduction.
// LDS of the per-bin interpolation: the window planes (real, imaginary), column-major,
// Gp[p * PL + c * PX + r]; PX = 8 mod 32 and PL = 16 mod 32 doubles make each A-operand load (8 rows
// x 4 columns x 2 planes) conflict-free.  4 columns beyond the 4 KS a bin needs: a group's steps
// start at its first column offset c0 and may run up to 3 columns past its last needed column
// c1 + 2 msp - 1 <= 15 + 2 msp - 1.  Then the nodes' fractional parts and stencil offsets.
template <int MSP>
struct Binterp2Lds {
    static constexpr int WX = 8 + 2 * MSP - 1, RBX = (WX + 7) / 8;
    static constexpr int WY = 16 + 2 * MSP - 1, KS = (WY + 3) / 4;
    static constexpr int NRW = 8 * RBX, NCW = 4 * KS + 4;
    static constexpr int PX = NRW + ((8 - NRW % 32) + 32) % 32;
    static constexpr int PL = NCW * PX + 16;
    static constexpr int bytes = 2 * PL * (int)sizeof(double) + kChunk * 2 * (int)sizeof(double) +
                                 kChunk * 2 * (int)sizeof(int);
};

// Start values of lane quarter ka's y-weight (columns c0 + 4 st + ka) and x-weight (rows 4 m + ka)
// recurrences for a node with fractional parts (d0, d1) and bin offsets (rx0, ry0) in a group whose
// first node has column offset c0: g = exp(-alpha x^2) at the first offset x, r = exp(-alpha (8 x + 16)).
template <int MSP>
__device__ __forceinline__ void binterp2_starts(double d0, double d1, int rx0, int ry0, int c0, int ka, double alpha,
                                                double2& wy, double2& wx) {
    const double y0 = (double)(c0 + ka - ry0 - (MSP - 1)) - d1;
    wy = make_double2(exp(-alpha * y0 * y0), exp(-alpha * (8.0 * y0 + 16.0)));
    const double x0 = (double)(ka - rx0 - (MSP - 1)) - d0;
    wx = make_double2(exp(-alpha * x0 * x0), exp(-alpha * (8.0 * x0 + 16.0)));
}

// The same for k_binterp2_32, whose lane quarter ka takes the x-weights of rows 4 (ka mod 2) + v
// (+ 8 rb) by a unit-step recurrence: r = exp(-alpha (2 x + 1)) at the first of them.
template <int MSP>
__device__ __forceinline__ void binterp2_32_starts(double d0, double d1, int rx0, int ry0, int c0, int ka, double alpha,
                                                   double2& wy, double2& wx) {
    const double y0 = (double)(c0 + ka - ry0 - (MSP - 1)) - d1;
    wy = make_double2(exp(-alpha * y0 * y0), exp(-alpha * (8.0 * y0 + 16.0)));
    const double x0 = (double)(4 * (ka & 1) - rx0 - (MSP - 1)) - d0;
    wx = make_double2(exp(-alpha * x0 * x0), exp(-alpha * (2.0 * x0 + 1.0)));
}

template <typename T, int MSP, bool ITAB = false>
__device__ __forceinline__ void binterp2_body(const V2<T>* __restrict__ grid, long long gstride, const NodeArgs& na,
                                              const EpiArgs& ea, double qq4, double2* __restrict__ zero,
                                              long long zero16, VBlk vb, unsigned char* smem) {
    using Lay = Binterp2Lds<MSP>;
    constexpr int RBX = Lay::RBX, KS = Lay::KS, NRW = Lay::NRW, NCW = Lay::NCW, PX = Lay::PX, PL = Lay::PL;
    double* Gp = reinterpret_cast<double*>(smem);
    double (*nd)[2] = reinterpret_cast<double (*)[2]>(smem + 2 * PL * sizeof(double));   // delta_0, delta_1
    int (*noff)[2] = reinterpret_cast<int (*)[2]>(smem + (2 * PL + 2 * kChunk) * sizeof(double));   // stencil starts
    // the spreading grid that follows is cleared here, a slice per workgroup, in the bandwidth this
    // compute-bound kernel leaves idle (16-byte stores)
    if (zero) {
        const long long nwg = (long long)vb.gx * vb.gy;
        const long long wg = (long long)vb.y * vb.gx + vb.x;
        const long long per = (zero16 + nwg - 1) / nwg;
        const long long e = min(zero16, (wg + 1) * per);
        for (long long i = wg * per + threadIdx.x; i < e; i += 256) zero[i] = make_double2(0.0, 0.0);
    }
    const int cid = split_id(na.csplit, vb.x);
    if (cid < 0) return;
    const Chunk ch = na.chunks[cid];
    const int b = vb.y;
    const int t = threadIdx.x;
    const V2<T>* g = grid + (long long)b * gstride;
    const int o0 = ch.t0 * 8 - (MSP - 1), o1 = ch.t1 * 16 - (MSP - 1);
    // lane quads read 4 adjacent columns of one row (64-byte segments); a wave covers 16 rows, so
    // its column-major LDS stores hit each bank at most twice
    // all of a thread's window loads are issued before the first LDS store
    constexpr int PER = (NRW * NCW + 255) / 256;
    V2<T> gv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = t + 256 * u;
        if (idx < NRW * NCW) {
            const int c = 4 * (idx / (4 * NRW)) + (idx & 3), r = (idx >> 2) % NRW;
            gv[u] = g[(long long)wrap(o0 + r, na.Mr[0]) * na.Mr[1] + wrap(o1 + c, na.Mr[1])];
        }
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = t + 256 * u;
        if (idx < NRW * NCW) {
            const int c = 4 * (idx / (4 * NRW)) + (idx & 3), r = (idx >> 2) % NRW;
            Gp[c * PX + r] = (double)gv[u].x;
            Gp[PL + c * PX + r] = (double)gv[u].y;
        }
    }
    if (t < ch.count) {
        const int node = ch.start + t;
        const double s0 = na.s[0][node], s1 = na.s[1][node];
        const double f0 = floor(s0), f1 = floor(s1);
        nd[t][0] = s0 - f0;
        nd[t][1] = s1 - f1;
        noff[t][0] = wrap((int)f0, na.Mr[0]) - ch.t0 * 8;    // in [0, 8)
        noff[t][1] = wrap((int)f1, na.Mr[1]) - ch.t1 * 16;   // in [0, 16)
    }
    __syncthreads();
    const int wv = t >> 6, lane = t & 63;
    const int ia = lane & 15, ka = lane >> 4;
    const double alpha = na.gc.alpha;
    const double* arow = &Gp[(ia >> 3) * PL + ka * PX + (ia & 7)];   // A operand: row block 0, column 0
    for (int k0 = 16 * wv; k0 < ch.count; k0 += 64) {
        const int jn = k0 + ia;
        // the chunk's nodes are ordered by column offset: the group's columns are
        // [c0, c1 + 2 msp), with c0, c1 the offsets of its first and last node
        const int c0 = noff[k0][1], c1 = noff[min(k0 + 15, ch.count - 1)][1];
        const int ksg = (c1 - c0 + 2 * MSP + 3) >> 2;   // k-steps this group needs (<= KS)
        double bv[KS], wx[2 * RBX];
        if (jn < ch.count) {
            const int rx0 = noff[jn][0], ry0 = noff[jn][1];
            double2 sy, sx;   // start values of the y- and x-weight recurrences
            if (ITAB) {   // the plan's table of these start values (fixed node positions)
                const double2* it2 = na.itab + 2 * (4 * (long long)(ch.start + jn) + ka);
                sy = it2[0];
                sx = it2[1];
            } else {
                binterp2_starts<MSP>(nd[jn][0], nd[jn][1], rx0, ry0, c0, ka, alpha, sy, sx);
            }
            {   // y-weights of columns c0 + 4 st + ka: stencil offset q = c0 + 4 st + ka - ry0 in [0, 2 msp)
                const int q0 = c0 + ka - ry0;
                double gg = sy.x, rr = sy.y;
#pragma unroll
                for (int st = 0; st < KS; ++st) {
                    const int q = q0 + 4 * st;
                    bv[st] = (q >= 0 && q < 2 * MSP) ? gg : 0.0;
                    gg *= rr;
                    rr *= qq4;
                }
            }
            {   // x-weights of rows 4 m + ka
                const int q0 = ka - rx0;
                double gg = sx.x, rr = sx.y;
#pragma unroll
                for (int m = 0; m < 2 * RBX; ++m) {
                    const int q = q0 + 4 * m;
                    wx[m] = (q >= 0 && q < 2 * MSP) ? gg : 0.0;
                    gg *= rr;
                    rr *= qq4;
                }
            }
        } else {
#pragma unroll
            for (int st = 0; st < KS; ++st) bv[st] = 0.0;
#pragma unroll
            for (int m = 0; m < 2 * RBX; ++m) wx[m] = 0.0;
        }
        // one accumulator per row block: independent product chains
        d4_t h[RBX];
#pragma unroll
        for (int rb = 0; rb < RBX; ++rb) h[rb] = d4_t{0.0, 0.0, 0.0, 0.0};
        const double* acol = arow + c0 * PX;
#pragma unroll
        for (int st = 0; st < KS; ++st) {
            if (st < ksg) {   // uniform over the wave
#pragma unroll
                for (int rb = 0; rb < RBX; ++rb)
                    h[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(acol[8 * rb + 4 * st * PX], bv[st], h[rb], 0, 0, 0);
            }
        }
        // register v of lane l holds H[i][l mod 16], i = 4 v + l / 16, within the row block:
        // (comp, x) = (0, ka), (0, 4 + ka), (1, ka), (1, 4 + ka); rows 8 rb + ka = 4 (2 rb) + ka
        double pre = 0.0, pim = 0.0;
#pragma unroll
        for (int rb = 0; rb < RBX; ++rb) {
            pre += wx[2 * rb] * h[rb][0] + wx[2 * rb + 1] * h[rb][1];
            pim += wx[2 * rb] * h[rb][2] + wx[2 * rb + 1] * h[rb][3];
        }
        pre += __shfl_xor(pre, 16);
        pim += __shfl_xor(pim, 16);
        pre += __shfl_xor(pre, 32);
        pim += __shfl_xor(pim, 32);
        if (ka == 0 && jn < ch.count) {
            const int node = ch.start + jn;
            epilogue<T>(ea, b, node, pre, pim, na.s[0][node], na.s[1][node]);
        }
    }
}

// (5 waves per SIMD where the LDS admits five workgroups per CU)
template <typename T, int MSP, bool ITAB>
__global__ void __launch_bounds__(256, Binterp2Lds<MSP>::bytes <= 32768 ? 5 : 3) k_binterp2(const V2<T>* __restrict__ grid, long long gstride,
                                                 NodeArgs na, EpiArgs ea, double qq4,
                                                 double2* __restrict__ zero, long long zero16) {
    __shared__ __align__(16) unsigned char smem[Binterp2Lds<MSP>::bytes];
    binterp2_body<T, MSP, ITAB>(grid, gstride, na, ea, qq4, zero, zero16, hw_block(), smem);
}

// The same per-bin interpolation on the FP32 matrix cores for FP32 plans: the window planes in LDS
// as FP32 (PX = 8 mod 32 floats, plane pitch PL = 32 mod 64 floats: the A-operand reads of a wave,
// 8 rows x 4 columns x 2 planes, then fall on distinct banks per half-wave), the nodes' y-weights
// from the same FP64 recurrence rounded to FP32, H = G B by v_mfma_f32_16x16x4f32 with FP32 sums
// over the <= KS column steps, and the contraction with the x-weights, the lane exchanges and the
// symbol epilogue in FP64.  Lane (ia, ka) holds H[4 ka + v][ia] in register v (rows (comp, x) =
// (ka / 2, 4 (ka mod 2) + v) of each 8-row block), so it needs the node's x-weights of rows
// 8 rb + 4 (ka mod 2) + v, taken from a unit-step Gaussian recurrence.
template <int MSP>
struct Binterp2Lds32 {
    static constexpr int WX = 8 + 2 * MSP - 1, RBX = (WX + 7) / 8;
    static constexpr int WY = 16 + 2 * MSP - 1, KS = (WY + 3) / 4;
    static constexpr int NRW = 8 * RBX, NCW = 4 * KS + 4;
    static constexpr int PX = NRW + ((8 - NRW % 32) + 32) % 32;
    static constexpr int PL0 = NCW * PX;
    static constexpr int PL = PL0 + ((32 - PL0 % 64) + 64) % 64;
    // the node tables first (8-byte aligned), then the FP32 window planes
    static constexpr int bytes = kChunk * 2 * (int)sizeof(double) + kChunk * 2 * (int)sizeof(int) +
                                 2 * PL * (int)sizeof(float);
};

template <int MSP, bool ITAB = false>
__device__ __forceinline__ void binterp2_32_body(const float2* __restrict__ grid, long long gstride, const NodeArgs& na,
                                                 const EpiArgs& ea, double qq4, double qq1, double2* __restrict__ zero,
                                                 long long zero16, VBlk vb, unsigned char* smem) {
    using Lay = Binterp2Lds32<MSP>;
    constexpr int RBX = Lay::RBX, KS = Lay::KS, NRW = Lay::NRW, NCW = Lay::NCW, PX = Lay::PX, PL = Lay::PL;
    double (*nd)[2] = reinterpret_cast<double (*)[2]>(smem);
    int (*noff)[2] = reinterpret_cast<int (*)[2]>(smem + kChunk * 2 * sizeof(double));
    float* Gp = reinterpret_cast<float*>(smem + kChunk * 2 * (sizeof(double) + sizeof(int)));
    if (zero) {
        const long long nwg = (long long)vb.gx * vb.gy;
        const long long wg = (long long)vb.y * vb.gx + vb.x;
        const long long per = (zero16 + nwg - 1) / nwg;
        const long long e = min(zero16, (wg + 1) * per);
        for (long long i = wg * per + threadIdx.x; i < e; i += 256) zero[i] = make_double2(0.0, 0.0);
    }
    const int cid = split_id(na.csplit, vb.x);
    if (cid < 0) return;
    const Chunk ch = na.chunks[cid];
    const int b = vb.y;
    const int t = threadIdx.x;
    const float2* g = grid + (long long)b * gstride;
    const int o0 = ch.t0 * 8 - (MSP - 1), o1 = ch.t1 * 16 - (MSP - 1);
    constexpr int PER = (NRW * NCW + 255) / 256;
    float2 gv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = t + 256 * u;
        if (idx < NRW * NCW) {
            const int c = 4 * (idx / (4 * NRW)) + (idx & 3), r = (idx >> 2) % NRW;
            gv[u] = g[(long long)wrap(o0 + r, na.Mr[0]) * na.Mr[1] + wrap(o1 + c, na.Mr[1])];
        }
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = t + 256 * u;
        if (idx < NRW * NCW) {
            const int c = 4 * (idx / (4 * NRW)) + (idx & 3), r = (idx >> 2) % NRW;
            Gp[c * PX + r] = gv[u].x;
            Gp[PL + c * PX + r] = gv[u].y;
        }
    }
    if (t < ch.count) {
        const int node = ch.start + t;
        const double s0 = na.s[0][node], s1 = na.s[1][node];
        const double f0 = floor(s0), f1 = floor(s1);
        nd[t][0] = s0 - f0;
        nd[t][1] = s1 - f1;
        noff[t][0] = wrap((int)f0, na.Mr[0]) - ch.t0 * 8;
        noff[t][1] = wrap((int)f1, na.Mr[1]) - ch.t1 * 16;
    }
    __syncthreads();
    const int wv = t >> 6, lane = t & 63;
    const int ia = lane & 15, ka = lane >> 4;
    const double alpha = na.gc.alpha;
    const float* arow = &Gp[(ia >> 3) * PL + ka * PX + (ia & 7)];
    const int xb = 4 * (ka & 1);   // first x row of this lane within each 8-row block
    for (int k0 = 16 * wv; k0 < ch.count; k0 += 64) {
        const int jn = k0 + ia;
        const int c0 = noff[k0][1], c1 = noff[min(k0 + 15, ch.count - 1)][1];
        const int ksg = (c1 - c0 + 2 * MSP + 3) >> 2;
        float bv[KS];
        double wx[RBX][4];
        if (jn < ch.count) {
            const int rx0 = noff[jn][0], ry0 = noff[jn][1];
            double2 sy, sx;   // start values of the y- and x-weight recurrences
            if (ITAB) {   // the plan's table of these start values (fixed node positions)
                const double2* it2 = na.itab + 2 * (4 * (long long)(ch.start + jn) + ka);
                sy = it2[0];
                sx = it2[1];
            } else {
                binterp2_32_starts<MSP>(nd[jn][0], nd[jn][1], rx0, ry0, c0, ka, alpha, sy, sx);
            }
            {   // y-weights of columns c0 + 4 st + ka
                const int q0 = c0 + ka - ry0;
                double gg = sy.x, rr = sy.y;
#pragma unroll
                for (int st = 0; st < KS; ++st) {
                    const int q = q0 + 4 * st;
                    bv[st] = (q >= 0 && q < 2 * MSP) ? (float)gg : 0.0f;
                    gg *= rr;
                    rr *= qq4;
                }
            }
            {   // x-weights of rows X = xb + 8 rb + v by the unit-step recurrence over X = xb .. 8 RBX - 1
                const int q0 = xb - rx0;
                double gg = sx.x, rr = sx.y;
#pragma unroll
                for (int rb = 0; rb < RBX; ++rb) {
#pragma unroll
                    for (int v = 0; v < 8; ++v) {
                        const int q = q0 + 8 * rb + v;
                        if (v < 4) wx[rb][v] = (q >= 0 && q < 2 * MSP) ? gg : 0.0;
                        gg *= rr;
                        rr *= qq1;
                    }
                }
            }
        } else {
#pragma unroll
            for (int st = 0; st < KS; ++st) bv[st] = 0.0f;
#pragma unroll
            for (int rb = 0; rb < RBX; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v) wx[rb][v] = 0.0;
        }
        f4_t h[RBX];
#pragma unroll
        for (int rb = 0; rb < RBX; ++rb) h[rb] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};
        const float* acol = arow + c0 * PX;
#pragma unroll
        for (int st = 0; st < KS; ++st) {
            if (st < ksg) {   // uniform over the wave
#pragma unroll
                for (int rb = 0; rb < RBX; ++rb)
                    h[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(acol[8 * rb + 4 * st * PX], bv[st], h[rb], 0, 0, 0);
            }
        }
        double part = 0.0;   // real part (ka < 2) or imaginary part (ka >= 2) of the node's sum
#pragma unroll
        for (int rb = 0; rb < RBX; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) part += wx[rb][v] * (double)h[rb][v];
        part += __shfl_xor(part, 16);
        const double pim = __shfl_down(part, 32);
        if (ka == 0 && jn < ch.count) {
            const int node = ch.start + jn;
            epilogue<float>(ea, b, node, part, pim, na.s[0][node], na.s[1][node]);
        }
    }
}

template <int MSP, bool ITAB>
__global__ void __launch_bounds__(256, 3) k_binterp2_32(const float2* __restrict__ grid, long long gstride,
                                                        NodeArgs na, EpiArgs ea, double qq4, double qq1,
                                                        double2* __restrict__ zero, long long zero16) {
    __shared__ __align__(16) unsigned char smem[Binterp2Lds32<MSP>::bytes];
    binterp2_32_body<MSP, ITAB>(grid, gstride, na, ea, qq4, qq1, zero, zero16, hw_block(), smem);
}

// ---- tile-gathered interpolation on the FP64 matrix cores -----------------------------------------
// For one gather tile with grid values G and a block of candidate nodes k, the part of the
// interpolation sum that the tile holds is
//   u_k = sum_x w0_k[x] H[x][k],   H[(comp, x)][k] = sum_j G_comp[x][j] B[j][k],
// with B[j][k] = w1_k[y] (2D, j = y) or w1_k[y] w2_k[z] (3D, j = 4y + z): H is a 16 x 16 x 16
// product for each group of 16 nodes (four v_mfma_f64_16x16x4 steps), the tile values G sit in
// registers as the A operand, B comes from LDS.  The contraction with w0 is a 4-term dot product
// per lane plus one lane exchange; the node's complex sum is added to its FP64 accumulator, which
// the per-node epilogue then turns into c_k (or rhohat_k).
// (5 waves per SIMD: 94-96 VGPRs, no spills; 4 waves were 10% slower at 256^3)
template <typename T, int MSP, int DIM>
__global__ void __launch_bounds__(2 * kMChunk, 5) k_minterp(const V2<T>* __restrict__ grid, long long gstride,
                                                        double2* __restrict__ acc, long long astride,
                                                        NodeArgs na, const GItem* __restrict__ items, int nitems,
                                                        const int* __restrict__ cand, double qq) {
    __shared__ double W1T[16][kMChunk];   // B operand, one row per tile column j
    __shared__ double W0T[8][kMChunk];    // w0 per tile row x
    __shared__ int nodes[kMChunk];
    const int iid = split_id(na.isplit);
    if (iid < 0) return;
    const GItem it = items[iid];
    const int b = blockIdx.y;
    const int t = threadIdx.x;
    const int o0 = it.g0 * 8;
    const int o1 = it.g1 * (DIM == 2 ? 16 : 4);
    const int o2 = it.g2 * 4;
    const int k = t & (kMChunk - 1);
    // A operand: lane l holds G_comp[x][j] for comp = (l mod 16) / 8, x = l mod 8, j = 4 s + l / 16
    const int wv = t >> 6, lane = t & 63;
    const int ia = lane & 15, ka = lane >> 4;
    const T* g = reinterpret_cast<const T*>(grid + (long long)b * gstride);
    double av[4];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        const int j = 4 * st + ka;
        const int x = o0 + (ia & 7);
        long long cell;
        if (DIM == 2)
            cell = (long long)x * na.Mr[1] + o1 + j;
        else
            cell = ((long long)x * na.Mr[1] + o1 + (j >> 2)) * na.Mr[2] + o2 + (j & 3);
        av[st] = (double)g[2 * cell + (ia >> 3)];
    }
    // node data of this thread's candidate in the current block, loaded one block ahead so that
    // the loads overlap the previous block's matrix products
    // (the candidate index one block further ahead, so that these loads do not wait for it)
    int fnode = 0;
    double fs = 0.0, fsb = 0.0;
    auto index_at = [&](int bs) -> int { return (bs + k < it.count) ? cand[it.start + bs + k] : 0; };
    auto fetch = [&](int bs, int node) {
        if (bs + k < it.count) {
            fnode = node;
            if (t < kMChunk) {
                fs = na.s[0][node];
            } else {
                fs = na.s[1][node];
                if (DIM == 3) fsb = na.s[2][node];
            }
        }
    };
    fetch(0, index_at(0));
    int nxt = index_at(kMChunk);
    for (int base = 0; base < it.count; base += kMChunk) {
        const int cnt = min(kMChunk, it.count - base);
        if (base > 0) __syncthreads();   // the previous block has read W0T, W1T and nodes
        const int node_c = fnode;
        const double s_c = fs, sb_c = fsb;
        if (t < kMChunk) {
            double w0[8];
#pragma unroll
            for (int x = 0; x < 8; ++x) w0[x] = 0.0;
            int node = 0;
            if (k < cnt) {
                node = node_c;
                tile_weights<MSP, 8>(s_c, o0, na.Mr[0], na.gc.alpha, qq, w0);
            }
            nodes[k] = node;
#pragma unroll
            for (int x = 0; x < 8; ++x) W0T[x][k] = w0[x];
        } else {
            double w1[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) w1[j] = 0.0;
            if (k < cnt) {
                if (DIM == 2) {
                    tile_weights<MSP, 16>(s_c, o1, na.Mr[1], na.gc.alpha, qq, w1);
                } else {
                    double a1[4], a2[4];
                    tile_weights<MSP, 4>(s_c, o1, na.Mr[1], na.gc.alpha, qq, a1);
                    tile_weights<MSP, 4>(sb_c, o2, na.Mr[2], na.gc.alpha, qq, a2);
#pragma unroll
                    for (int y = 0; y < 4; ++y)
#pragma unroll
                        for (int z = 0; z < 4; ++z) w1[4 * y + z] = a1[y] * a2[z];
                }
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) W1T[j][k] = w1[j];
        }
        __syncthreads();
        fetch(base + kMChunk, nxt);
        nxt = index_at(base + 2 * kMChunk);
#pragma unroll
        for (int gi = 0; gi < kMChunk / 64; ++gi) {
            const int k0 = 16 * (wv + 4 * gi);
            if (k0 >= cnt) break;
            d4_t hacc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int st = 0; st < 4; ++st)
                hacc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[st], W1T[4 * st + ka][k0 + ia], hacc, 0, 0, 0);
            // register v of lane l holds H[i][k0 + l mod 16] with i = 4 v + l / 16, i.e.
            // (comp, x) = (0, ka), (0, 4 + ka), (1, ka), (1, 4 + ka) for v = 0..3
            const double wa = W0T[ka][k0 + ia], wb = W0T[4 + ka][k0 + ia];
            double pre = wa * hacc[0] + wb * hacc[1];
            double pim = wa * hacc[2] + wb * hacc[3];
            pre += __shfl_xor(pre, 16);
            pim += __shfl_xor(pim, 16);
            pre += __shfl_xor(pre, 32);
            pim += __shfl_xor(pim, 32);
            if (ka < 2 && k0 + ia < cnt) {
                double* dst = reinterpret_cast<double*>(acc + (long long)b * astride + nodes[k0 + ia]) + ka;
                global_add<double>(dst, ka == 0 ? pre : pim);
            }
        }
    }
}

// per-node epilogue of the tile-gathered interpolation
template <typename T>
__global__ void k_iepilogue(const double2* __restrict__ acc, long long astride, long long Mh, NodeArgs na,
                            EpiArgs ea) {
    const int b = blockIdx.y;
    for (long long node = (long long)blockIdx.x * blockDim.x + threadIdx.x; node < Mh;
         node += (long long)gridDim.x * blockDim.x) {
        const double2 v = acc[(long long)b * astride + node];
        epilogue<T>(ea, b, (int)node, v.x, v.y, na.s[0][node], na.s[1][node]);
    }
}

template <typename T>
__global__ void k_fill_one(V2<T>* c, long long count) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
        c[i] = mk2<T>((T)1, (T)0);
}

// ---- fold of a caller-supplied full node vector (type-1 stage entry) ---------------------------
// Re sum_all c_m e^{ikx} = Re sum_half (c_m + conj(c_{-m})) e^{ikx}
template <typename T>
__global__ void k_fold(const V2<T>* __restrict__ c, long long cstride, V2<T>* __restrict__ cbuf, long long Mh,
                       const int* __restrict__ perm, int hphi, int n_phi, int n_theta) {
    const int b = blockIdx.y;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < Mh; i += (long long)gridDim.x * blockDim.x) {
        int hm = perm[i];
        int ab = hm / hphi, cc = hm - ab * hphi;
        long long m = (long long)ab * n_phi + cc;
        long long mp;
        if (n_theta == 1) mp = m + hphi;
        else {
            int a = ab / n_theta, bb = ab - a * n_theta;
            mp = ((long long)a * n_theta + (n_theta - 1 - bb)) * n_phi + cc + hphi;
        }
        V2<T> x = c[(long long)b * cstride + m], y = c[(long long)b * cstride + mp];
        cbuf[(long long)b * Mh + i] = mk2<T>(x.x + y.x, x.y - y.y);
    }
}

// ---- FP64 moments of the density (2D Laplace subtraction, Alg. 1 first step) -------------------
// Argument records of the stencil bodies for the persistent executor.
struct BinterpTask {
    const void* grid;
    long long gstride;
    NodeArgs na;
    EpiArgs ea;
    double qq4, qq1;
    double2* zero;
    long long zero16;
};
struct MspreadTask {
    void* grid;
    long long gstride;
    const void* cbuf;
    long long cstride;
    NodeArgs na;
    const GItem* items;
    int nitems;
    const int* cand;
    double qq;
    BinArgs ba;
};

}  // namespace nlf
