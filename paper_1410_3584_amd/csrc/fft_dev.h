// Device code of the Stockham FFT (kernel bodies and their launch wrappers); the host launchers
// are in fft.hip.  Included by fft.hip and by solvers.hip (the persistent executor).
#pragma once
#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "exec.h"
#include "nlf_internal.h"

namespace nlf {

template <typename T> __device__ __forceinline__ V2<T> mk(T x, T y);
template <> __device__ __forceinline__ float2 mk<float>(float x, float y) { return make_float2(x, y); }
template <> __device__ __forceinline__ double2 mk<double>(double x, double y) { return make_double2(x, y); }

template <typename T> __device__ __forceinline__ V2<T> cadd(V2<T> a, V2<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ V2<T> csub(V2<T> a, V2<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ V2<T> cmul(V2<T> a, V2<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Elements held in LDS per workgroup and threads per workgroup.  The strided-axis kernel keeps
// C adjacent columns (128 KiB in both precisions) so that row segments load contiguously; the
// contiguous-axis kernel needs no such block and keeps at most 2048 elements (one or two long
// lines), which gives many small workgroups per CU.
template <typename T> struct FftCfg;
template <> struct FftCfg<double> { static constexpr int E = 8192, NT = 512; };
template <> struct FftCfg<float>  { static constexpr int E = 16384, NT = 1024; };
struct RowCfg { static constexpr int E = 2048, NT = 512; };
// Strided-axis kernel for short columns (n <= 512): half the LDS of FftCfg, so that two workgroups
// share a CU, and 1024 threads, so that each thread has few loads in flight (measured at 256^3:
// 256 threads 7.3 ms per split potential, 512 threads 6.5 ms, 1024 threads 6.2 ms).
struct ColSmallCfg { static constexpr int E = 4096, NT = 1024; };
// The passes of lines up to 512 points as the persistent executor runs them: 256 threads and
// element budgets that give each thread as many elements as the kernels' own configurations.
struct ExecRowCfg { static constexpr int E = 1024, NT = 256; };
struct ExecColCfg { static constexpr int E = 1024, NT = 256; };
// 1024-point lines held in LDS (the oversampled axes of the 512^2 grids; the 2D rows and the columns
// now take the register-resident kernels of fft.hip, these shapes the lines those do not cover).
// Measured at 512^2 with the LDS kernels on both axes (FP64 evaluation, forward + inverse FFT
// stages, us): these shapes 26.7 + 23.3; rows of 128 or 1024 threads per
// line 27.4-32.9 + 25.3-26.6 (a pass has 128 radix-8 butterflies per line, but the 512 line
// workgroups then hold too few waves per CU to cover the loads); twiddles in LDS 27.4 + 25.0;
// column blocks of 2 columns (256 threads) or of 4 with 1024 threads 27.3-27.9 + 25.2-27.0.
struct Row1024Cfg { static constexpr int E = 1024, NT = 512; static constexpr bool TWL = false; };
struct Col1024Cfg { static constexpr int E = 8192, NT = 512; static constexpr bool TWL = false; };

// data index j (0..nd-1, x_j = -L + j h) -> row of the 2x oversampled periodic grid holding
// centred frequency/position j - nd/2
__device__ __forceinline__ int dmap(int j, int nd, int Mr) {
    int c = j - nd / 2;
    return c < 0 ? c + Mr : c;
}
__device__ __forceinline__ bool is_data_row(int r, int nd, int Mr) { return r < nd / 2 || r >= Mr - nd / 2; }

// In-place multi-line Stockham FFT of nl lines of length n = 2^lg held in buf[line*pitch + lpad<HALF>(i)].
// tw[t] = exp(-2 pi i t / n).  DIR = -1 forward, +1 inverse (unnormalised).  Mixed radix: one radix-2 or radix-4 pass first when lg is not a multiple of 3, then radix-8
// passes, each a read of the whole buffer into registers and a write back (fewer LDS round trips
// than radix 4: 512 points take 3 passes instead of 5).  Pass with radix R over the index range
// q = n / R, after p = product of the earlier radices: butterfly i (k = i mod p) reads
// x[i + m q], m < R, scales element m by w^(m k n / (R p)), takes the length-R DFT and writes
// element m to x[(i - k) R + k + m p].
template <typename T, int DIR>
__device__ __forceinline__ void dft4(V2<T>& a0, V2<T>& a1, V2<T>& a2, V2<T>& a3) {
    const V2<T> t0 = cadd<T>(a0, a2), t1 = csub<T>(a0, a2), t2 = cadd<T>(a1, a3), t3 = csub<T>(a1, a3);
    a0 = cadd<T>(t0, t2);
    a2 = csub<T>(t0, t2);
    if (DIR < 0) {
        a1 = mk<T>(t1.x + t3.y, t1.y - t3.x);
        a3 = mk<T>(t1.x - t3.y, t1.y + t3.x);
    } else {
        a1 = mk<T>(t1.x - t3.y, t1.y + t3.x);
        a3 = mk<T>(t1.x + t3.y, t1.y - t3.x);
    }
}

// length-8 DFT in place: even and odd halves by dft4, combined with w8^k = exp(DIR 2 pi i k / 8)
template <typename T, int DIR>
__device__ __forceinline__ void dft8(V2<T> (&a)[8]) {
    dft4<T, DIR>(a[0], a[2], a[4], a[6]);
    dft4<T, DIR>(a[1], a[3], a[5], a[7]);
    const T h = (T)0.70710678118654752440;
    // odd part times w8^k, k = 0..3 (a[1], a[3], a[5], a[7] hold O_0..O_3)
    V2<T> o1 = a[3], o2 = a[5], o3 = a[7];
    if (DIR < 0) {
        o1 = mk<T>(h * (o1.x + o1.y), h * (o1.y - o1.x));     // (1 - i)/sqrt2
        o2 = mk<T>(o2.y, -o2.x);                               // -i
        o3 = mk<T>(h * (o3.y - o3.x), -h * (o3.x + o3.y));    // (-1 - i)/sqrt2
    } else {
        o1 = mk<T>(h * (o1.x - o1.y), h * (o1.y + o1.x));     // (1 + i)/sqrt2
        o2 = mk<T>(-o2.y, o2.x);                               // i
        o3 = mk<T>(-h * (o3.x + o3.y), h * (o3.x - o3.y));    // (-1 + i)/sqrt2
    }
    const V2<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6], o0 = a[1];
    a[0] = cadd<T>(e0, o0);
    a[4] = csub<T>(e0, o0);
    a[1] = cadd<T>(e1, o1);
    a[5] = csub<T>(e1, o1);
    a[2] = cadd<T>(e2, o2);
    a[6] = csub<T>(e2, o2);
    a[3] = cadd<T>(e3, o3);
    a[7] = csub<T>(e3, o3);
}

// LDS position of element e of a line, PAD: one padding slot after every 8 elements.  A radix-8
// pass writes 8 consecutive outputs per thread (the first pass) or runs of 8 (the second);
// unpadded, the lanes of a wave then hit the same few banks (16-byte elements 128 bytes apart),
// padded they spread.  The column kernels pad lines of up to 512 points (256^3: fused axis-0
// kernel 928 -> 821 us, axis-1 passes 218/213 -> 202/194 us), which is exactly when their twiddles
// are staged in LDS (TWL); the 1024-point columns of the 2D grids are not padded (padded, a 512^2
// evaluation took 4.5% longer), nor are the row kernels (their 512-point lines took 209 -> 226 us
// padded: the larger LDS footprint costs a workgroup per CU).
template <bool PAD>
__device__ __forceinline__ int lpad(int e) { return PAD ? e + (e >> 3) : e; }
__host__ __device__ __forceinline__ int lds_line(int n, bool pad) { return pad ? n + (n >> 3) : n; }

// All sizes are powers of two (lg = log2 n, lgp = log2 p): indices by shifts and masks.
template <typename T, int DIR, int NT, int E, int R, bool HALF, bool PAD>
__device__ __forceinline__ void fft_pass(V2<T>* buf, int pitch, int n, int lg, int nl, int p, int lgp,
                                         const V2<T>* __restrict__ tw) {
    constexpr int RB = (E + R * NT - 1) / (R * NT);   // butterflies per thread
    constexpr int LR = R == 2 ? 1 : (R == 4 ? 2 : 3);
    const int lq = lg - LR;                            // q = n / R
    const int q = 1 << lq;
    const int tot = nl << lq;
    const int lts = lq - lgp;                          // tstep = n / (R p)
    const int tid = threadIdx.x;
    V2<T> y[RB][R];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int idx = tid + r * NT;
        if (idx < tot) {
            const int line = idx >> lq, i = idx & (q - 1);
            const int k = i & (p - 1);
            const V2<T>* x = buf + line * pitch;
#pragma unroll
            for (int m = 0; m < R; ++m) y[r][m] = x[lpad<PAD>(i + m * q)];
            if (p > 1) {
#pragma unroll
                for (int m = 1; m < R; ++m) {
                    const int tt = (m * k) << lts;
                    V2<T> w;
                    if constexpr (HALF) {   // half table (in LDS): w^(t + n/2) = -w^t
                        w = tw[tt < (n >> 1) ? tt : tt - (n >> 1)];
                        if (tt >= (n >> 1)) { w.x = -w.x; w.y = -w.y; }
                    } else {
                        w = tw[tt];
                    }
                    if (DIR > 0) w.y = -w.y;
                    y[r][m] = cmul<T>(y[r][m], w);
                }
            }
            if constexpr (R == 2) {
                const V2<T> a0 = y[r][0], a1 = y[r][1];
                y[r][0] = cadd<T>(a0, a1);
                y[r][1] = csub<T>(a0, a1);
            } else if constexpr (R == 4) {
                dft4<T, DIR>(y[r][0], y[r][1], y[r][2], y[r][3]);
            } else {
                static_assert(R == 8, "radix 2, 4 or 8");
                dft8<T, DIR>(y[r]);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int idx = tid + r * NT;
        if (idx < tot) {
            const int line = idx >> lq, i = idx & (q - 1);
            const int k = i & (p - 1);
            const int j = (i - k) * R + k;
            V2<T>* x = buf + line * pitch;
#pragma unroll
            for (int m = 0; m < R; ++m) x[lpad<PAD>(j + m * p)] = y[r][m];
        }
    }
    __syncthreads();
}

// HALF: tw holds w^t for t < n/2 only (the LDS copy); otherwise the full table
template <typename T, int DIR, int NT, int E, bool HALF = false, bool PAD = HALF>
__device__ void lds_fft(V2<T>* buf, int pitch, int n, int lg, int nl, const V2<T>* __restrict__ tw) {
    int p = 1, lgp = 0;
    if (lg % 3 == 1) {
        fft_pass<T, DIR, NT, E, 2, HALF, PAD>(buf, pitch, n, lg, nl, p, lgp, tw);
        p = 2;
        lgp = 1;
    } else if (lg % 3 == 2) {
        fft_pass<T, DIR, NT, E, 4, HALF, PAD>(buf, pitch, n, lg, nl, p, lgp, tw);
        p = 4;
        lgp = 2;
    }
    while (p < n) {
        fft_pass<T, DIR, NT, E, 8, HALF, PAD>(buf, pitch, n, lg, nl, p, lgp, tw);
        p *= 8;
        lgp += 3;
    }
}

// ---- contiguous-axis kernel ---------------------------------------------------------------------
enum { LOAD_GRID = 0, LOAD_RHO = 1 };
enum { STORE_GRID = 0, STORE_U = 1 };

struct RowsArgs {
    void* grid;            // complex lines of length n
    long long gstride;     // batch stride of grid (elements)
    const void* rho;       // LOAD_RHO: real data [batch][N]
    void* u;               // STORE_U: real output [batch][N]
    long long rstride;     // batch stride of rho / u (elements)
    int n, lg;             // FFT length along the last axis and log2
    int nlines;            // active lines per batch field
    int lines_per_wg;
    int dim;
    int nd[3], Mr[3];      // data and oversampled sizes (for the mapped modes)
    const double* dec0; const double* dec1; const double* dec2;  // 1/c_g per axis (mapped modes)
    const void* tw;
    double post;           // output scale (STORE_U)
    int accum;             // STORE_U: add to u instead of overwriting it
    int band;              // > 0: only the cells |f| < band of a line are nonzero / needed (the
                           // ball of a split): LOAD_GRID reads only those, STORE_GRID writes only those
    int half;              // > 0: a grid line holds the first `half` (> n/2) outputs of a transform of
                           // real data, line pitch `half`: STORE_GRID writes those, LOAD_GRID
                           // rebuilds the rest from the Hermitian symmetry v[n - c] = conj v[c]
    // 2D Laplace: u += m0 u11 - m1 . u12 (Sec. 2.2, Eqs. 'phi1_exct', 'phi12_ext')
    int add_u1;
    const double* mom;     // [batch][4]: m0, m1x, m1y
    const double* u11;     // [N]: u_{1,1} on the grid
    double sigma, L0, L1, h0, h1;
    // LOAD_RHO, 2D Laplace: per-workgroup partial sums of rho, x rho, y rho ([batch][grid.x][3])
    double* mom_part;
    int* nonfinite;        // LOAD_RHO: set to 1 when a density value is NaN or +-Inf (may be NULL)
};

// sum of v over the workgroup (blockDim.x a multiple of 64, <= 1024); every thread gets it
__device__ __forceinline__ double wg_sum(double v, double* sh16) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh16[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += sh16[i];
    return s;
}

// TWL: the twiddle table is staged in LDS (short lines, n <= 512) or read from global memory
// through the L1 cache (longer lines: measured faster for the 1024-point columns of the 2D grids)
template <typename T, typename TIO, int DIR, int LOAD, int STORE, int E, bool TWL, int NT>
__device__ __forceinline__ void fft_rows_body(const RowsArgs& a, VBlk vb, unsigned char* smem_raw) {
    V2<T>* buf = reinterpret_cast<V2<T>*>(smem_raw);
    const int n = a.n;
    const int pitch = n;   // rows are not padded (see lpad)
    const int b = vb.y;
    const int line0 = vb.x * a.lines_per_wg;
    const int nl = min(a.lines_per_wg, a.nlines - line0);
    V2<T>* grid = reinterpret_cast<V2<T>*>(a.grid) + (long long)b * a.gstride;
    const bool mapped = (LOAD == LOAD_RHO) || (STORE == STORE_U);
    const int last = a.dim - 1;
    const int ndl = a.nd[last];

    // grid line index and the per-line deconvolution factor of line (line0 + l)
    auto grid_line = [&](int l, double* fac, int* j0o, int* j1o) -> long long {
        int al = line0 + l;
        if (!mapped) return al;
        if (a.dim == 2) {
            *j0o = al; *j1o = 0;
            *fac = a.dec0[al];
            return dmap(al, a.nd[0], a.Mr[0]);
        }
        int j0 = al / a.nd[1], j1 = al - j0 * a.nd[1];
        *j0o = j0; *j1o = j1;
        *fac = a.dec0[j0] * a.dec1[j1];
        return (long long)dmap(j0, a.nd[0], a.Mr[0]) * a.Mr[1] + dmap(j1, a.nd[1], a.Mr[1]);
    };
    const double* decl = (a.dim == 2) ? a.dec1 : a.dec2;
    // the line's twiddle table, staged in LDS after the data (read by every FFT pass)
    V2<T>* twl = buf + a.lines_per_wg * pitch;
    constexpr int PERT = (E + NT - 1) / NT;
    V2<T> tv[PERT];
#pragma unroll
    for (int u = 0; u < PERT; ++u) {
        const int i = threadIdx.x + u * NT;
        if (TWL && i < (n >> 1)) tv[u] = reinterpret_cast<const V2<T>*>(a.tw)[i];
    }

    // ---- load
    if (LOAD == LOAD_RHO) {
        const TIO* rho = reinterpret_cast<const TIO*>(a.rho) + (long long)b * a.rstride;
        double m0 = 0.0, mx = 0.0, my = 0.0;   // moments of the rows read (2D Laplace)
        // every load of the thread is issued before the first use (one memory latency, not PER)
        constexpr int PER = (E + NT - 1) / NT;
        double rv[PER], dv[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int idx = threadIdx.x + u * NT;
            rv[u] = 0.0;
            dv[u] = 0.0;
            if (idx < nl * n) {
                const int l = idx >> a.lg, c = idx & (n - 1);
                // oversampled position c holds data index j with dmap(j) == c, if any
                if (is_data_row(c, ndl, n)) {
                    const int j = (c < ndl / 2) ? c + ndl / 2 : c - (n - ndl / 2);
                    rv[u] = (double)rho[(long long)(line0 + l) * ndl + j];
                    dv[u] = decl[j];
                }
            }
        }
        if (a.nonfinite) {   // a NaN or Inf anywhere in the density: flag the plan (rare path)
            bool bad = false;
#pragma unroll
            for (int u = 0; u < PER; ++u) bad = bad || !isfinite(rv[u]);
            if (bad) atomicOr(a.nonfinite, 1);
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int idx = threadIdx.x + u * NT;
            if (idx < nl * n) {
                const int l = idx >> a.lg, c = idx & (n - 1);
                double fac = 1;
                int j0 = 0, j1 = 0;
                (void)grid_line(l, &fac, &j0, &j1);
                V2<T> v = mk<T>(0, 0);
                if (is_data_row(c, ndl, n)) {
                    const int j = (c < ndl / 2) ? c + ndl / 2 : c - (n - ndl / 2);
                    v.x = (T)(rv[u] * fac * dv[u]);
                    if (a.mom_part) {
                        m0 += rv[u];
                        mx += rv[u] * (-a.L0 + (line0 + l) * a.h0);
                        my += rv[u] * (-a.L1 + j * a.h1);
                    }
                }
                buf[l * pitch + c] = v;
            }
        }
        if (a.mom_part) {   // uniform over the workgroup
            __shared__ double red16[16];
            m0 = wg_sum(m0, red16);
            mx = wg_sum(mx, red16);
            my = wg_sum(my, red16);
            if (threadIdx.x == 0) {
                double* o = a.mom_part + ((long long)b * vb.gx + vb.x) * 3;
                o[0] = m0;
                o[1] = mx;
                o[2] = my;
            }
        }
    } else {
        constexpr int PER = (E + NT - 1) / NT;
        V2<T> v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int idx = threadIdx.x + u * NT;
            v[u] = mk<T>(0, 0);
            if (idx < nl * n) {
                const int l = idx >> a.lg, c = idx & (n - 1);
                double fac;
                int j0, j1;
                const long long gl = grid_line(l, &fac, &j0, &j1);
                if (a.half) {
                    const bool lo = c <= (n >> 1);
                    const V2<T> w = grid[gl * a.half + (lo ? c : n - c)];
                    v[u] = lo ? w : mk<T>(w.x, -w.y);
                } else if (!a.band || is_data_row(c, 2 * a.band, n)) {
                    v[u] = grid[gl * n + c];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int idx = threadIdx.x + u * NT;
            if (idx < nl * n) buf[(idx >> a.lg) * pitch + (idx & (n - 1))] = v[u];
        }
    }
#pragma unroll
    for (int u = 0; u < PERT; ++u) {
        const int i = threadIdx.x + u * NT;
        if (TWL && i < (n >> 1)) twl[i] = tv[u];
    }
    __syncthreads();
    lds_fft<T, DIR, NT, E, TWL, false>(buf, pitch, n, a.lg, nl, TWL ? twl : reinterpret_cast<const V2<T>*>(a.tw));

    // ---- store
    if (STORE == STORE_GRID && a.half) {
        for (int idx = threadIdx.x; idx < nl * a.half; idx += NT) {
            int l = idx / a.half, c = idx - l * a.half;
            double fac;
            int j0, j1;
            long long gl = grid_line(l, &fac, &j0, &j1);
            grid[gl * a.half + c] = buf[l * pitch + c];
        }
    } else if (STORE == STORE_GRID) {
        for (int idx = threadIdx.x; idx < nl * n; idx += NT) {
            int l = idx >> a.lg, c = idx & (n - 1);
            double fac;
            int j0, j1;
            long long gl = grid_line(l, &fac, &j0, &j1);
            if (!a.band || is_data_row(c, 2 * a.band, n)) grid[gl * n + c] = buf[l * pitch + c];
        }
    } else {
        TIO* u = reinterpret_cast<TIO*>(a.u) + (long long)b * a.rstride;
        double m0 = 0, m1x = 0, m1y = 0;
        if (a.add_u1) {
            m0 = a.mom[4 * b + 0];
            m1x = a.mom[4 * b + 1];
            m1y = a.mom[4 * b + 2];
        }
        const double inv2s2 = 1.0 / (2.0 * a.sigma * a.sigma);
        const int lgd = __builtin_ctz(ndl);   // the data length is a power of two (half the line)
        for (int idx = threadIdx.x; idx < nl * ndl; idx += NT) {
            int l = idx >> lgd, j = idx & (ndl - 1);
            double fac;
            int j0, j1;
            (void)grid_line(l, &fac, &j0, &j1);
            int c = dmap(j, ndl, n);
            double val = (double)buf[l * pitch + c].x * fac * decl[j] * a.post;
            if (a.add_u1) {
                // 2D only: line = row j0, element j = column index
                // u_{1,2} = -(x/|x|^2)(1 - e^{-|x|^2/(2 sigma^2)})/(2 pi), 0 at x = 0 (Eq. 'phi12_ext')
                double x = -a.L0 + j0 * a.h0, y = -a.L1 + j * a.h1;
                double r2 = x * x + y * y;
                double f = (r2 > 0) ? expm1(-r2 * inv2s2) / (2.0 * 3.14159265358979323846 * r2) : 0.0;
                val += m0 * a.u11[(long long)j0 * ndl + j] - (m1x * f * x + m1y * f * y);
            }
            TIO* dst = u + (long long)(line0 + l) * ndl + j;
            *dst = a.accum ? (TIO)((double)*dst + val) : (TIO)val;
        }
    }
}

template <typename T, typename TIO, int DIR, int LOAD, int STORE, int E, bool TWL, int NT = RowCfg::NT>
__global__ void __launch_bounds__(NT) k_fft_rows(RowsArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    fft_rows_body<T, TIO, DIR, LOAD, STORE, E, TWL, NT>(a, hw_block(), smem_raw);
}

// ---- strided-axis kernel ----------------------------------------------------------------------
struct ColsArgs {
    void* grid;
    long long gstride;      // batch stride (elements)
    int n, lg;              // FFT length along this axis
    long long inner;        // elements between consecutive rows of a line (product of later axes)
    int C;                  // adjacent columns per workgroup (divides inner)
    int ncb;                // column blocks per outer index = inner / C
    int outer_mapped;       // 1: outer index o is a data index of the previous axis (pruned)
    int outer_nd, outer_Mr;
    int nd;                 // data count along this axis (for pruning)
    int nd_store;           // > 0: SPRUNE keeps rows |f| < nd_store / 2 instead of nd
    // > 0: only the columns of a band are transformed (the ball of a split): c2 with |f2| < bc2 of
    // the innermost axis (length Mr2), and, for the axis-0 pass, c1 with |f1| < bc1 (length Mr1)
    int bc1, bc2, Mr1, Mr2;
    const void* tw;
    // optional: workgroup (0, 0, b) reduces the moment partials of the row pass for field b
    const double* mom_part;
    int mom_nblk;
    double mom_w;           // cell volume
    double* mom;            // [batch][4]: m0, m1x, m1y, 0
};

// first column of column block cb: consecutive blocks of C columns, or, with a band, the blocks of
// the band's columns (c2 in [0, bc2) and [Mr2 - bc2, Mr2); for the axis-0 pass also c1 likewise)
__device__ __forceinline__ long long band_col(const ColsArgs& a, int cb) {
    if (!a.bc2) return (long long)cb * a.C;
    const int nb2 = 2 * a.bc2 / a.C;
    const int i1 = cb / nb2, j = cb - i1 * nb2;
    int c2 = j * a.C;
    c2 = c2 < a.bc2 ? c2 : a.Mr2 - 2 * a.bc2 + c2;
    if (!a.bc1) return c2;
    const int c1 = i1 < a.bc1 ? i1 : a.Mr1 - 2 * a.bc1 + i1;
    return (long long)c1 * a.Mr2 + c2;
}

// 2D Laplace: one workgroup of the forward column pass adds the row pass's per-workgroup partial
// sums of rho, x rho, y rho of field z into its moments m0, m1 (uniform over the workgroup)
__device__ __forceinline__ void finish_moments(const ColsArgs& a, int z, int nt) {
    __shared__ double red16[16];
    const double* part = a.mom_part + (long long)z * a.mom_nblk * 3;
    double s[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < a.mom_nblk; i += nt)
        for (int k = 0; k < 3; ++k) s[k] += part[3 * i + k];
    for (int k = 0; k < 3; ++k) s[k] = wg_sum(s[k], red16);
    if (threadIdx.x == 0) {
        double* m = a.mom + 4 * z;
        m[0] = a.mom_w * s[0];
        m[1] = a.mom_w * s[1];
        m[2] = a.mom_w * s[2];
        m[3] = 0.0;
    }
}

template <typename T, int DIR, bool LPRUNE, bool SPRUNE, int NT, int E, bool TWL>
__device__ __forceinline__ void fft_cols_body(const ColsArgs& a, VBlk vb, unsigned char* smem_raw) {
    V2<T>* buf = reinterpret_cast<V2<T>*>(smem_raw);
    const int n = a.n, C = a.C, lgC = __builtin_ctz(C);   // C is a power of two
    const int pitch = lds_line(n, TWL) + 1;
    if (a.mom && vb.x == 0 && vb.y == 0) finish_moments(a, vb.z, NT);   // uniform over the workgroup
    // XCD-aware order: consecutive hardware workgroup ids go round-robin over the 8 XCDs; give
    // each XCD a contiguous range of column blocks so neighbouring row segments share its L2.
    int cb = vb.x;
    const int nb = vb.gx;
    if ((nb & 7) == 0) cb = (cb & 7) * (nb >> 3) + (cb >> 3);
    int o = vb.y;
    long long go = a.outer_mapped ? dmap(o, a.outer_nd, a.outer_Mr) : o;
    V2<T>* base = reinterpret_cast<V2<T>*>(a.grid) + (long long)vb.z * a.gstride +
                  go * (long long)n * a.inner + band_col(a, cb);
    // every load of the thread (data and the twiddle table, which is staged in LDS after the
    // data) is issued before the first LDS write: one memory latency, not PER
    constexpr int PER = (E + NT - 1) / NT;
    V2<T> v[PER], tv[PER];
    V2<T>* twl = buf + C * pitch;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = threadIdx.x + u * NT;
        v[u] = mk<T>(0, 0);
        if (idx < n * C) {
            const int r = idx >> lgC, c = idx & (C - 1);
            if (!LPRUNE || is_data_row(r, a.nd, n)) v[u] = base[(long long)r * a.inner + c];
        }
        if (TWL && idx < (n >> 1)) tv[u] = reinterpret_cast<const V2<T>*>(a.tw)[idx];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = threadIdx.x + u * NT;
        if (idx < n * C) buf[(idx & (C - 1)) * pitch + lpad<TWL>(idx >> lgC)] = v[u];
        if (TWL && idx < (n >> 1)) twl[idx] = tv[u];
    }
    __syncthreads();
    lds_fft<T, DIR, NT, E, TWL>(buf, pitch, n, a.lg, C, TWL ? twl : reinterpret_cast<const V2<T>*>(a.tw));
    const int nds = a.nd_store > 0 ? a.nd_store : a.nd;
    for (int idx = threadIdx.x; idx < n * C; idx += NT) {
        int r = idx >> lgC, c = idx & (C - 1);
        if (!SPRUNE || is_data_row(r, nds, n)) base[(long long)r * a.inner + c] = buf[c * pitch + lpad<TWL>(r)];
    }
}

template <typename T, int DIR, bool LPRUNE, bool SPRUNE, int NT, int E, bool TWL>
__global__ void __launch_bounds__(NT) k_fft_cols(ColsArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    fft_cols_body<T, DIR, LPRUNE, SPRUNE, NT, E, TWL>(a, hw_block(), smem_raw);
}

// Fused axis-0 pass of a split's I1 (Eq. '3.9'): per column (c1, c2) of the padded spectrum (axes
// 1 and 2 already transformed), the forward FFT of the n0 data rows, the multiply by
// w(k) = (1 - e^{-|k|^2/a}) / |k|^2 (w(0) = 1/a), the inverse FFT, and the store of the n0 data rows
// only: the full Mr0-row spectrum never goes to memory.
struct ConvW {
    int Mr0, Mr1, Mr2;
    int pitch2;            // stored columns of the innermost axis (its first pitch2 frequencies)
    double dk0, dk1, dk2, inva;
    const double* e0;      // exp(-k0^2 / a) per axis-0 frequency row (the register kernel)
};

// 1/x for normal x > 0: the hardware estimate refined by two Newton steps (within an ulp or two of
// the quotient, not correctly rounded)
__device__ __forceinline__ double rcp_newton(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

template <typename T, int NT, int E, bool TWL>
__global__ void __launch_bounds__(NT) k_fft_conv0(ColsArgs a, ConvW cw) {
    static_assert(NT % 16 == 0, "a thread keeps one of the C <= 16 columns");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V2<T>* buf = reinterpret_cast<V2<T>*>(smem_raw);
    const int n = a.n, C = a.C, lgC = __builtin_ctz(C);   // C is a power of two
    const int pitch = lds_line(n, TWL) + 1;
    int cb = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0) cb = (cb & 7) * (nb >> 3) + (cb >> 3);
    const long long col0 = (long long)cb * C;
    V2<T>* base = reinterpret_cast<V2<T>*>(a.grid) + (long long)blockIdx.z * a.gstride + col0;
    constexpr int PER = (E + NT - 1) / NT;
    V2<T> v[PER], tv[PER];
    V2<T>* twl = buf + C * pitch;   // twiddles staged in LDS after the data
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = threadIdx.x + u * NT;
        v[u] = mk<T>(0, 0);
        if (idx < n * C) {
            const int r = idx >> lgC, c = idx & (C - 1);
            if (is_data_row(r, a.nd, n)) v[u] = base[(long long)r * a.inner + c];
        }
        if (TWL && idx < (n >> 1)) tv[u] = reinterpret_cast<const V2<T>*>(a.tw)[idx];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = threadIdx.x + u * NT;
        if (idx < n * C) buf[(idx & (C - 1)) * pitch + lpad<TWL>(idx >> lgC)] = v[u];
        if (TWL && idx < (n >> 1)) twl[idx] = tv[u];
    }
    __syncthreads();
    lds_fft<T, -1, NT, E, TWL>(buf, pitch, n, a.lg, C, TWL ? twl : reinterpret_cast<const V2<T>*>(a.tw));
    __syncthreads();
    // a thread keeps one column (NT is a multiple of C): its (k1, k2) part once, and
    // e^{-|k|^2/a} = e^{-k0^2/a} e^{-(k1^2 + k2^2)/a}; near k = 0, where 1 - e^{-x} cancels, expm1
    const int c = threadIdx.x & (C - 1);
    const long long col = col0 + c;
    const int c1 = (int)(col / cw.pitch2), c2 = (int)(col - (long long)c1 * cw.pitch2);
    const double k1 = (c1 < cw.Mr1 / 2 ? c1 : c1 - cw.Mr1) * cw.dk1;
    const double k2 = (c2 < cw.Mr2 / 2 ? c2 : c2 - cw.Mr2) * cw.dk2;
    const double q12 = k1 * k1 + k2 * k2;
    const double e12 = exp(-q12 * cw.inva);
    for (int idx = threadIdx.x; idx < n * C; idx += NT) {
        const int r = idx >> lgC;
        const double k0 = (r < cw.Mr0 / 2 ? r : r - cw.Mr0) * cw.dk0;
        const double kk = k0 * k0 + q12;
        const double x = kk * cw.inva;
        double w;
        if (x >= 1.0) w = (1.0 - exp(-k0 * k0 * cw.inva) * e12) / kk;
        else w = kk > 0.0 ? -expm1(-x) / kk : cw.inva;
        V2<T> e = buf[c * pitch + lpad<TWL>(r)];
        e.x = (T)((double)e.x * w);
        e.y = (T)((double)e.y * w);
        buf[c * pitch + lpad<TWL>(r)] = e;
    }
    __syncthreads();
    lds_fft<T, 1, NT, E, TWL>(buf, pitch, n, a.lg, C, TWL ? twl : reinterpret_cast<const V2<T>*>(a.tw));
    __syncthreads();
    for (int idx = threadIdx.x; idx < n * C; idx += NT) {   // column c of this thread, as above
        const int r = idx >> lgC;
        if (is_data_row(r, a.nd, n)) base[(long long)r * a.inner + c] = buf[c * pitch + lpad<TWL>(r)];
    }
}


}  // namespace nlf
