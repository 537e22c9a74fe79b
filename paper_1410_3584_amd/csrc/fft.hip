// Hand-written Stockham FFT for gfx950, used on the 2x-oversampled NUFFT grid and on the
// solver grid.  One workgroup transforms a block of lines held in LDS (radix-8 passes, after one
// radix-2 or radix-4 pass when log2 n is not a multiple of 3).  Two kernels:
//   k_fft_rows : lines along the contiguous (last) axis.  Optional fused prologue/epilogue:
//                real density in -> precorrect (divide by the Gaussian's Fourier coefficients)
//                and zero-pad into the oversampled line (type-2 NUFFT input), and
//                oversampled line -> truncate, postcorrect, real part (+ the analytic u1 term of
//                the 2D Laplace kernel) -> potential out (type-1 NUFFT output).
//   k_fft_cols : lines along a strided axis, C adjacent columns per workgroup so each row
//                segment is a contiguous load; optional pruning of the zero rows on load (the
//                padded half of the type-2 input) and of the unused rows on store (the half of the
//                type-1 output that is cut away).
// The NUFFT sums these feed are those of Sec. 2.1, Eq. 'ifft'.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "fft_dev.h"

namespace nlf {

template <typename T>
__global__ void k_fill_zero(T* p, long long count) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long st = (long long)gridDim.x * blockDim.x;
    for (; i < count; i += st) p[i] = (T)0;
}

// 16-byte stores, four per thread and pass (the bulk of a 16-byte aligned buffer)
__global__ void k_fill_zero16(double2* p, long long count) {
    const long long st = (long long)gridDim.x * blockDim.x;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const double2 z = make_double2(0.0, 0.0);
    for (; i + 3 * st < count; i += 4 * st) {
        p[i] = z;
        p[i + st] = z;
        p[i + 2 * st] = z;
        p[i + 3 * st] = z;
    }
    for (; i < count; i += st) p[i] = z;
}

// ---- host launchers ---------------------------------------------------------------------------
static int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// Task kinds of the FFT passes the persistent executor runs (lines of up to 512 points, the
// 2048-element row budget and the short-column configuration, twiddles in LDS), or -1.
template <typename T, typename TIO, int DIR, int LOAD, int STORE, int E, bool TWL>
static constexpr int rows_kind() {
    constexpr bool d = std::is_same<T, double>::value, f = std::is_same<T, float>::value;
    if (E != ExecRowCfg::E || !TWL) return -1;
    if (LOAD == LOAD_RHO && STORE == STORE_GRID && DIR < 0 && std::is_same<T, TIO>::value)
        return d ? TK_ROWS_RHO_D : TK_ROWS_RHO_F;
    if (LOAD == LOAD_GRID && STORE == STORE_U && DIR > 0 && d)
        return std::is_same<TIO, double>::value ? TK_ROWS_U_D : TK_ROWS_U_DF;
    if (LOAD == LOAD_GRID && STORE == STORE_GRID && std::is_same<T, TIO>::value && (d || f))
        return DIR < 0 ? (d ? TK_ROWS_FWD_D : TK_ROWS_FWD_F) : (d ? TK_ROWS_INV_D : TK_ROWS_INV_F);
    return -1;
}
template <typename T, int DIR, bool LP, bool SP, int NT, int E, bool TWL>
static constexpr int cols_kind() {
    constexpr bool d = std::is_same<T, double>::value;
    if (NT != ExecColCfg::NT || E != ExecColCfg::E || !TWL) return -1;
    if (LP && !SP && DIR < 0) return d ? TK_COLS_PFWD_D : TK_COLS_PFWD_F;
    if (!LP && SP && DIR > 0) return d ? TK_COLS_PINV_D : -1;
    if (!LP && !SP) return DIR < 0 ? (d ? TK_COLS_FWD_D : TK_COLS_FWD_F) : (d ? TK_COLS_INV_D : TK_COLS_INV_F);
    return -1;
}

template <typename T, int DIR, int LOAD, int STORE, typename TIO, int E, bool TWL, int NT = RowCfg::NT>
static int launch_rows_cfg(nlf_plan* p, RowsArgs a, int batch) {
    a.lg = ilog2(a.n);
    a.lines_per_wg = std::max(1, E / a.n);
    if (a.n > E) return set_error(NLF_EUNSUPPORTED, "FFT length %d exceeds the LDS line budget", a.n);
    dim3 grid((a.nlines + a.lines_per_wg - 1) / a.lines_per_wg, batch);
    size_t lds = ((size_t)a.lines_per_wg * a.n + (TWL ? a.n / 2 : 0)) * sizeof(V2<T>);   // lines (+ twiddles)
    if (Recorder* rec = recorder()) {
        constexpr int kind = rows_kind<T, TIO, DIR, LOAD, STORE, E, TWL>();
        if (kind < 0 || a.half || a.band || a.accum) {
            rec->failed = 1;
            return NLF_OK;
        }
        return record(rec, kind, grid, lds, a);
    }
    // raised on first need; the check and the raise are one step, for plans driven from several threads
    static std::mutex attr_mu;
    static size_t attr_bytes = 0;
    {
        std::lock_guard<std::mutex> lock(attr_mu);
        if (lds > attr_bytes) {
            NLF_HIP(hipFuncSetAttribute((const void*)&k_fft_rows<T, TIO, DIR, LOAD, STORE, E, TWL, NT>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            attr_bytes = lds;
        }
    }
    hipLaunchKernelGGL((k_fft_rows<T, TIO, DIR, LOAD, STORE, E, TWL, NT>), grid, dim3(NT), lds, p->stream, a);
    NLF_HIP(hipGetLastError());
    return NLF_OK;
}

// Contiguous-axis pass of 1024-point lines of a 2D grid with the lines in registers (the passes of
// k_fft_cols_r): L lines per workgroup, 128 threads per line, thread t holding the elements
// t + 128 m of its line, so that a wave's loads and stores are contiguous.  The fused prologue and
// epilogue are those of fft_rows_body for 2D lines: LOAD_RHO reads the density's data row into the
// oversampled positions with the precorrection (and the Laplace moments' partial sums, and the
// non-finite check), STORE_U writes the data positions of the real part with the postcorrection
// (and the analytic u1 of the Laplace kernel); LOAD_GRID / STORE_GRID move whole lines.
template <typename T, typename TIO, int DIR, int LOAD, int STORE, int L>
__global__ void __launch_bounds__(L * 128) k_fft_rows_r(RowsArgs a) {
    constexpr int LG = 10, N = 1 << LG, Q = N / 8;
    constexpr int PITCH = N + (N >> 3) + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V2<T>* buf = reinterpret_cast<V2<T>*>(smem_raw);
    V2<T>* tw = buf + L * PITCH;   // half twiddle table
    const int tid = threadIdx.x;
    const int l = tid / Q, t = tid % Q;
    const int b = blockIdx.y;
    const int al = blockIdx.x * L + l;   // data line (row j0 of the 2D data grid when mapped)
    const bool valid = al < a.nlines;
    constexpr bool mapped = (LOAD == LOAD_RHO) || (STORE == STORE_U);
    const int ndl = a.nd[1];
    const long long gl = mapped ? dmap(valid ? al : 0, a.nd[0], a.Mr[0]) : al;
    const double fac = (mapped && valid) ? a.dec0[al] : 1.0;
    V2<T>* grid = reinterpret_cast<V2<T>*>(a.grid) + (long long)b * a.gstride;
    V2<T> x[8];
    if (LOAD == LOAD_RHO) {
        const TIO* rho = reinterpret_cast<const TIO*>(a.rho) + (long long)b * a.rstride + (long long)al * ndl;
        double m0 = 0.0, mx = 0.0, my = 0.0;
        double rv[8], dv[8];   // every load issued before the first use
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int c = t + m * Q;
            rv[m] = 0.0;
            dv[m] = 0.0;
            if (valid && is_data_row(c, ndl, N)) {   // oversampled position c holds data index j
                const int j = (c < ndl / 2) ? c + ndl / 2 : c - (N - ndl / 2);
                rv[m] = (double)rho[j];
                dv[m] = a.dec1[j];
            }
        }
        bool bad = false;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int c = t + m * Q;
            const int j = (c < ndl / 2) ? c + ndl / 2 : c - (N - ndl / 2);
            bad = bad || !isfinite(rv[m]);
            x[m] = mk<T>((T)(rv[m] * fac * dv[m]), 0);
            if (a.mom_part && is_data_row(c, ndl, N)) {
                m0 += rv[m];
                mx += rv[m] * (-a.L0 + al * a.h0);
                my += rv[m] * (-a.L1 + j * a.h1);
            }
        }
        if (a.nonfinite && bad) atomicOr(a.nonfinite, 1);
        if (a.mom_part) {   // uniform over the workgroup
            __shared__ double red16[16];
            m0 = wg_sum(m0, red16);
            mx = wg_sum(mx, red16);
            my = wg_sum(my, red16);
            if (tid == 0) {
                double* o = a.mom_part + ((long long)b * gridDim.x + blockIdx.x) * 3;
                o[0] = m0;
                o[1] = mx;
                o[2] = my;
            }
        }
    } else {
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m] = valid ? grid[gl * N + t + m * Q] : mk<T>(0, 0);
    }
    // STORE_U: the epilogue's per-element factors, loaded before the transform
    double pv[8], uv[8], m0 = 0, m1x = 0, m1y = 0;
    if (STORE == STORE_U) {
        if (a.add_u1) {
            m0 = a.mom[4 * b + 0];
            m1x = a.mom[4 * b + 1];
            m1y = a.mom[4 * b + 2];
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int c = t + m * Q;
            const int j = (c < ndl / 2) ? c + ndl / 2 : c - (N - ndl / 2);
            pv[m] = 0.0;
            uv[m] = 0.0;
            if (valid && is_data_row(c, ndl, N)) {
                pv[m] = a.dec1[j];
                if (a.add_u1) uv[m] = a.u11[(long long)al * ndl + j];
            }
        }
    }
    for (int i = tid; i < N / 2; i += L * Q) tw[i] = reinterpret_cast<const V2<T>*>(a.tw)[i];
    V2<T>* line = buf + l * PITCH;
    __syncthreads();   // twiddles staged
    // radix 2 (p = 1) on the registers m, m + 4, then three radix-8 passes (as in k_fft_cols_r)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const V2<T> u = x[m], v = x[m + 4];
        const int i = t + m * Q;
        line[lpad<true>(2 * i)] = cadd<T>(u, v);
        line[lpad<true>(2 * i + 1)] = csub<T>(u, v);
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 8; ++m) x[m] = line[lpad<true>(t + m * Q)];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int lgp = 1 + 3 * s, p = 1 << lgp, k = t & (p - 1);
        const int lts = LG - 3 - lgp;
#pragma unroll
        for (int m = 1; m < 8; ++m) {
            const int tt = (m * k) << lts;
            V2<T> w = tw[tt < N / 2 ? tt : tt - N / 2];
            if (tt >= N / 2) { w.x = -w.x; w.y = -w.y; }
            if (DIR > 0) w.y = -w.y;
            x[m] = cmul<T>(x[m], w);
        }
        dft8<T, DIR>(x);
        if (s < 2) {
            const int j = (t - k) * 8 + k;
            __syncthreads();
#pragma unroll
            for (int m = 0; m < 8; ++m) line[lpad<true>(j + m * p)] = x[m];
            __syncthreads();
#pragma unroll
            for (int m = 0; m < 8; ++m) x[m] = line[lpad<true>(t + m * Q)];
        }
    }
    if (!valid) return;
    if (STORE == STORE_GRID) {
#pragma unroll
        for (int m = 0; m < 8; ++m) grid[gl * N + t + m * Q] = x[m];
    } else {
        TIO* u = reinterpret_cast<TIO*>(a.u) + (long long)b * a.rstride + (long long)al * ndl;
        const double inv2s2 = 1.0 / (2.0 * a.sigma * a.sigma);
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int c = t + m * Q;
            if (!is_data_row(c, ndl, N)) continue;
            const int j = (c < ndl / 2) ? c + ndl / 2 : c - (N - ndl / 2);
            double val = (double)x[m].x * fac * pv[m] * a.post;
            if (a.add_u1) {   // u_{1,2} as in fft_rows_body (Eq. 'phi12_ext')
                const double xx = -a.L0 + al * a.h0, yy = -a.L1 + j * a.h1;
                const double r2 = xx * xx + yy * yy;
                const double f = (r2 > 0) ? expm1(-r2 * inv2s2) / (2.0 * 3.14159265358979323846 * r2) : 0.0;
                val += m0 * uv[m] - (m1x * f * xx + m1y * f * yy);
            }
            u[j] = a.accum ? (TIO)((double)u[j] + val) : (TIO)val;
        }
    }
}

// Contiguous-axis pass of lines of N = 64 to 512 points with the lines in registers, the lines of
// a wave inside the wave: lane (l, t), l < 512 / N, holds the elements t + m N/8 of line l, so the
// exchanges between the passes (a first radix-2 or radix-4 pass when log2 N is not a multiple of 3,
// then radix-8 passes) stay inside the wave and need no workgroup barrier, only the wave's own LDS
// writes to have completed.  The exchanges move the real and the imaginary parts in turn through
// lines of scalars (half the LDS of complex lines, so more resident workgroups).  W waves per
// workgroup share the staged twiddle table.  The fused modes are those of fft_rows_body: LOAD_RHO
// (density row with the precorrection), STORE_U (the data positions of the real part with the
// postcorrection, optionally added to u), the Hermitian half of a transform of real data (STORE_GRID
// writes the first `half` outputs, LOAD_GRID rebuilds the rest) and the band of a split's ball (only
// |f| < band read or written).  The mapped modes take data lines of half the line length.
__device__ __forceinline__ void wave_lds_sync() { __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// LDS of k_fft_rows_rw: per wave 512/N scalar lines of N + N/8 + 1 entries, then the half twiddle table
template <typename T, int LG, int W> constexpr size_t rows_rw_tw_offset() {
    return ((size_t)W * (512 >> LG) * ((1 << LG) + (1 << (LG - 3)) + 1) * sizeof(T) + 15) / 16 * 16;
}
template <typename T, int LG, int W> constexpr size_t rows_rw_lds() {
    return rows_rw_tw_offset<T, LG, W>() + (size_t)(1 << (LG - 1)) * 2 * sizeof(T);
}

template <typename T, typename TIO, int DIR, int LOAD, int STORE, int LG, int W>
__global__ void __launch_bounds__(W * 64) k_fft_rows_rw(RowsArgs a) {
    constexpr int N = 1 << LG, Q = N / 8, LPW = 64 / Q, R2 = LG % 3, NP = LG / 3;
    constexpr int PITCH = N + (N >> 3) + 1;
    static_assert(LG >= 6 && LG <= 9, "64 to 512 points");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* buf = reinterpret_cast<T*>(smem_raw);
    V2<T>* tw = reinterpret_cast<V2<T>*>(smem_raw + rows_rw_tw_offset<T, LG, W>());   // half twiddle table
    const int tid = threadIdx.x;
    const int wv = tid >> 6, lane = tid & 63;
    const int t = lane % Q;
    const int b = blockIdx.y;
    const int al = (blockIdx.x * W + wv) * LPW + lane / Q;   // data line (j0 nd1 + j1 in 3D) when mapped
    const bool valid = al < a.nlines;
    constexpr bool mapped = (LOAD == LOAD_RHO) || (STORE == STORE_U);
    const int last = a.dim - 1;
    const int ndl = a.nd[last];
    const double* decl = (a.dim == 2) ? a.dec1 : a.dec2;
    long long gl = al;
    double fac = 1.0;
    if (mapped) {
        const int la = valid ? al : 0;
        if (a.dim == 2) {
            gl = dmap(la, a.nd[0], a.Mr[0]);
            fac = a.dec0[la];
        } else {
            const int j0 = la / a.nd[1], j1 = la - j0 * a.nd[1];
            gl = (long long)dmap(j0, a.nd[0], a.Mr[0]) * a.Mr[1] + dmap(j1, a.nd[1], a.Mr[1]);
            fac = a.dec0[j0] * a.dec1[j1];
        }
    }
    V2<T>* grid = reinterpret_cast<V2<T>*>(a.grid) + (long long)b * a.gstride;
    V2<T> x[8];
    // mapped modes: the data line is half the line, so the data positions t + Q m are those of
    // m = 0, 1 (data index c + N/4) and m = 6, 7 (c - 3N/4)
    constexpr int DM[4] = {0, 1, 6, 7};
    auto data_j = [&](int m) { const int c = t + m * Q; return m < 2 ? c + N / 4 : c - 3 * N / 4; };
    if (LOAD == LOAD_RHO) {
        const TIO* rho = reinterpret_cast<const TIO*>(a.rho) + (long long)b * a.rstride + (long long)al * ndl;
        double rv[4], dv[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const int j = data_j(DM[d]);
            rv[d] = valid ? (double)rho[j] : 0.0;
            dv[d] = decl[j];
        }
        bool bad = false;
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m] = mk<T>(0, 0);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            bad = bad || !isfinite(rv[d]);
            x[DM[d]].x = (T)(rv[d] * fac * dv[d]);
        }
        if (a.nonfinite && bad) atomicOr(a.nonfinite, 1);
    } else if (a.half) {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int c = t + m * Q;
            const bool lo = c <= (N >> 1);
            x[m] = mk<T>(0, 0);
            if (valid) {
                const V2<T> w = grid[gl * a.half + (lo ? c : N - c)];
                x[m] = lo ? w : mk<T>(w.x, -w.y);
            }
        }
    } else {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int c = t + m * Q;
            x[m] = (valid && (!a.band || is_data_row(c, 2 * a.band, N))) ? grid[gl * N + c] : mk<T>(0, 0);
        }
    }
    // STORE_U: the values added to, loaded before the transform
    double uo[4] = {0.0, 0.0, 0.0, 0.0};
    if (STORE == STORE_U && a.accum && valid) {
        const TIO* u = reinterpret_cast<const TIO*>(a.u) + (long long)b * a.rstride + (long long)al * ndl;
#pragma unroll
        for (int d = 0; d < 4; ++d) uo[d] = (double)u[data_j(DM[d])];
    }
    for (int i = tid; i < N / 2; i += W * 64) tw[i] = reinterpret_cast<const V2<T>*>(a.tw)[i];
    T* line = buf + (wv * LPW + lane / Q) * PITCH;
    __syncthreads();   // twiddles staged; from here on each wave works alone
    // y[m] goes to position pos[m] of the line; the next pass reads t + Q m
    auto exchange = [&](const V2<T> (&y)[8], const int (&pos)[8]) {
        wave_lds_sync();   // the wave's reads of the previous exchange are done
#pragma unroll
        for (int m = 0; m < 8; ++m) line[lpad<true>(pos[m])] = y[m].x;
        wave_lds_sync();   // and its writes of this one
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m].x = line[lpad<true>(t + m * Q)];
        wave_lds_sync();
#pragma unroll
        for (int m = 0; m < 8; ++m) line[lpad<true>(pos[m])] = y[m].y;
        wave_lds_sync();
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m].y = line[lpad<true>(t + m * Q)];
    };
    if constexpr (R2 == 1) {   // radix 2, p = 1: butterfly i = t + Q m (m < 4) on x[i], x[i + N/2]
        V2<T> y[8];
        int pos[8];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int i = t + m * Q;
            y[m] = cadd<T>(x[m], x[m + 4]);
            y[m + 4] = csub<T>(x[m], x[m + 4]);
            pos[m] = 2 * i;
            pos[m + 4] = 2 * i + 1;
        }
        exchange(y, pos);
    } else if constexpr (R2 == 2) {   // radix 4, p = 1: butterfly i = t + Q m (m < 2) on x[i + k N/4]
        V2<T> y[8];
        int pos[8];
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            V2<T> a0 = x[m], a1 = x[m + 2], a2 = x[m + 4], a3 = x[m + 6];
            dft4<T, DIR>(a0, a1, a2, a3);
            const int i = t + m * Q;
            y[m] = a0;
            y[m + 2] = a1;
            y[m + 4] = a2;
            y[m + 6] = a3;
            pos[m] = 4 * i;
            pos[m + 2] = 4 * i + 1;
            pos[m + 4] = 4 * i + 2;
            pos[m + 6] = 4 * i + 3;
        }
        exchange(y, pos);
    }
#pragma unroll
    for (int s = 0; s < NP; ++s) {
        const int lgp = R2 + 3 * s, p = 1 << lgp, k = t & (p - 1);
        if (p > 1) {
            const int lts = LG - 3 - lgp;   // twiddle stride N / (8 p)
#pragma unroll
            for (int m = 1; m < 8; ++m) {
                const int tt = (m * k) << lts;
                V2<T> w = tw[tt < N / 2 ? tt : tt - N / 2];
                if (tt >= N / 2) { w.x = -w.x; w.y = -w.y; }
                if (DIR > 0) w.y = -w.y;
                x[m] = cmul<T>(x[m], w);
            }
        }
        dft8<T, DIR>(x);
        if (s + 1 < NP) {
            const int j = (t - k) * 8 + k;
            V2<T> y[8];
            int pos[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                y[m] = x[m];
                pos[m] = j + m * p;
            }
            exchange(y, pos);
        }
    }
    if (!valid) return;
    if (STORE == STORE_GRID) {
#pragma unroll
        for (int m = 0; m < 8; ++m) {   // outputs t + Q m
            const int c = t + m * Q;
            if (a.half) {
                if (c < a.half) grid[gl * a.half + c] = x[m];
            } else if (!a.band || is_data_row(c, 2 * a.band, N)) {
                grid[gl * N + c] = x[m];
            }
        }
    } else {
        TIO* u = reinterpret_cast<TIO*>(a.u) + (long long)b * a.rstride + (long long)al * ndl;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const int j = data_j(DM[d]);
            u[j] = (TIO)(uo[d] + (double)x[DM[d]].x * fac * decl[j] * a.post);
        }
    }
}

// waves per workgroup of k_fft_rows_rw.  Measured at 256^3 (FP64 split potential, the four
// 512-point row passes, us): complex exchanges 117 + 113 + 102 + 133, the real and imaginary parts
// in turn (7 resident workgroups instead of 3) 85 + 82 + 81 + 114.
constexpr int kRowsW = 4;

template <typename T, int DIR, int LOAD, int STORE, typename TIO, int LG>
static int launch_rows_rw(nlf_plan* p, RowsArgs a, int batch) {
    constexpr int LPWG = kRowsW * (512 >> LG);   // lines per workgroup
    a.lg = LG;
    a.lines_per_wg = LPWG;
    dim3 grid((a.nlines + LPWG - 1) / LPWG, batch);
    const size_t lds = rows_rw_lds<T, LG, kRowsW>();   // <= 23 KiB
    hipLaunchKernelGGL((k_fft_rows_rw<T, TIO, DIR, LOAD, STORE, LG, kRowsW>), grid, dim3(kRowsW * 64), lds, p->stream, a);
    NLF_HIP(hipGetLastError());
    return NLF_OK;
}

// rows of 64 to 512 points take k_fft_rows_rw: not the 2D moments or u1 terms, and in the mapped
// modes only data lines of half the line
static bool rows_rw_applies(const RowsArgs& a, bool mapped) {
    return a.n >= 64 && a.n <= 512 && (a.dim == 2 || a.dim == 3) && !a.mom_part && !a.add_u1 &&
           (!mapped || 2 * a.nd[a.dim - 1] == a.n);
}

// lines per workgroup of k_fft_rows_r.  Measured at 512^2 (FP64 evaluation, forward + inverse
// FFT stages, us): one line per workgroup 20.1-20.5 + 19.9-20.2, two 20.7-20.8 + 19.0-19.2, the
// LDS-resident rows (k_fft_rows) 22.1 + 19.7-19.8.
constexpr int kRowsRL = 1;   // the forward pass (LOAD_RHO), which also sums moments per workgroup
template <int LOAD> constexpr int rows_r_lines() { return LOAD == LOAD_RHO ? kRowsRL : 2; }

template <typename T, int DIR, int LOAD, int STORE, typename TIO>
static int launch_rows_r(nlf_plan* p, RowsArgs a, int batch) {
    constexpr int N = 1024, LPW = rows_r_lines<LOAD>();
    a.lg = 10;
    a.lines_per_wg = LPW;
    dim3 grid((a.nlines + LPW - 1) / LPW, batch);
    const size_t lds = ((size_t)LPW * (N + (N >> 3) + 1) + N / 2) * sizeof(V2<T>);   // <= 45 KiB
    hipLaunchKernelGGL((k_fft_rows_r<T, TIO, DIR, LOAD, STORE, LPW>), grid, dim3(LPW * 128), lds, p->stream, a);
    NLF_HIP(hipGetLastError());
    return NLF_OK;
}

// rows of 1024 points of 2D grids (no Hermitian half, no band) take k_fft_rows_r
static bool rows_r_applies(const RowsArgs& a) { return a.n == 1024 && a.dim == 2 && !a.half && !a.band; }

// LDS element budget of the contiguous-axis kernel for lines of length n: 1024-point lines get
// one line per workgroup (twice the workgroups of the 2048-element budget)
static int rows_budget(int n) { return n == 1024 ? Row1024Cfg::E : RowCfg::E; }
// lines per workgroup of the 2D row pass (the Laplace moments' partial sums are per workgroup)
static int rows_lines_per_wg(int n) { return n == 1024 ? kRowsRL : std::max(1, rows_budget(n) / n); }

template <typename T, int DIR, int LOAD, int STORE, typename TIO = T>
static int launch_rows(nlf_plan* p, RowsArgs a, int batch) {
    if (recorder() && a.n <= 512)   // recorded for the persistent executor
        return launch_rows_cfg<T, DIR, LOAD, STORE, TIO, ExecRowCfg::E, true>(p, a, batch);
    if (!recorder() && rows_r_applies(a)) return launch_rows_r<T, DIR, LOAD, STORE, TIO>(p, a, batch);
    if (!recorder() && rows_rw_applies(a, LOAD == LOAD_RHO || STORE == STORE_U)) {
        switch (a.n) {
            case 512: return launch_rows_rw<T, DIR, LOAD, STORE, TIO, 9>(p, a, batch);
            case 256: return launch_rows_rw<T, DIR, LOAD, STORE, TIO, 8>(p, a, batch);
            case 128: return launch_rows_rw<T, DIR, LOAD, STORE, TIO, 7>(p, a, batch);
            case 64: return launch_rows_rw<T, DIR, LOAD, STORE, TIO, 6>(p, a, batch);
            default: break;
        }
    }
    if (a.n == 1024)
        return launch_rows_cfg<T, DIR, LOAD, STORE, TIO, Row1024Cfg::E, Row1024Cfg::TWL, Row1024Cfg::NT>(p, a, batch);
    if (a.n <= 512) return launch_rows_cfg<T, DIR, LOAD, STORE, TIO, RowCfg::E, true>(p, a, batch);
    return launch_rows_cfg<T, DIR, LOAD, STORE, TIO, RowCfg::E, false>(p, a, batch);
}

template <typename T, int DIR, bool LP, bool SP, int NT, int E, bool TWL>
static int launch_cols_cfg(nlf_plan* p, ColsArgs a, int outer, int batch) {
    a.lg = ilog2(a.n);
    // C adjacent columns per workgroup: as many as the element budget E allows (the padded pitch
    // n + 1 adds at most C <= 16 elements of LDS), wider row segments coalesce better, but not so
    // many that fewer than 256 workgroups remain (one per CU)
    auto blocks = [&](int c) -> long long {
        return (a.bc2 ? (long long)(a.bc1 ? 2 * a.bc1 : 1) * (2 * a.bc2 / c) : a.inner / c) * outer * batch;
    };
    int C = 16;
    while (C > 1 && (C * a.n > E || a.inner % C || blocks(C) < 256)) C >>= 1;
    if (a.n + 1 > E) return set_error(NLF_EUNSUPPORTED, "FFT length %d exceeds the LDS line budget", a.n);
    a.C = C;
    if (a.bc2 && (a.bc2 % C || 2 * a.bc2 > (a.bc1 ? a.Mr2 : a.inner) || (a.bc1 && 2 * a.bc1 > a.Mr1)))
        return set_error(NLF_EINVAL, "column band %d/%d does not fit the grid", a.bc1, a.bc2);
    a.ncb = a.bc2 ? (a.bc1 ? 2 * a.bc1 : 1) * (2 * a.bc2 / C) : (int)(a.inner / C);
    dim3 grid(a.ncb, outer, batch);
    size_t lds = ((size_t)C * (lds_line(a.n, TWL) + 1) + (TWL ? a.n / 2 : 0)) * sizeof(V2<T>);   // columns (+ twiddles)
    if (Recorder* rec = recorder()) {
        constexpr int kind = cols_kind<T, DIR, LP, SP, NT, E, TWL>();
        if (kind < 0 || a.bc2) {
            rec->failed = 1;
            return NLF_OK;
        }
        return record(rec, kind, grid, lds, a);
    }
    // raised on first need; the check and the raise are one step, for plans driven from several threads
    static std::mutex attr_mu;
    static size_t attr_bytes = 0;
    {
        std::lock_guard<std::mutex> lock(attr_mu);
        if (lds > attr_bytes) {
            NLF_HIP(hipFuncSetAttribute((const void*)&k_fft_cols<T, DIR, LP, SP, NT, E, TWL>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            attr_bytes = lds;
        }
    }
    hipLaunchKernelGGL((k_fft_cols<T, DIR, LP, SP, NT, E, TWL>), grid, dim3(NT), lds, p->stream, a);
    NLF_HIP(hipGetLastError());
    return NLF_OK;
}

// w^tt (0 <= tt < n = 2^LG) from the quarter table w^t, t < n/4, of w = e^{-2 pi i/n}:
// w^(t + n/4) = -i w^t.  The register-resident column kernels stage only this quarter: at 1024
// points the half table pushed a workgroup's LDS just past a half (FP64) or a quarter (FP32, and the
// 512-point fused axis-0 kernel) of the CU's 160 KiB, one resident workgroup fewer.
template <typename T, int LG>
__device__ __forceinline__ V2<T> qtw(const V2<T>* tw, int tt) {
    V2<T> w = tw[tt & ((1 << (LG - 2)) - 1)];
    const int q = tt >> (LG - 2);
    if (q & 1) w = mk<T>(w.y, -w.x);
    if (q & 2) w = mk<T>(-w.x, -w.y);
    return w;
}

// Strided-axis pass of n = 2^LG-point lines with the lines in registers, for n = 512 = 8 x 8 x 8
// and n = 1024 = 2 x 8 x 8 x 8 (the oversampled axes of the 256^3 and 512^2 grids).  Thread t of a
// column holds the 8 elements t + m n/8 (m = 0..7).  With a radix-2 factor, its registers m and
// m + 4 are the two inputs of the first pass's butterflies t + m n/8 (m < 4); then radix-8
// passes, one butterfly per thread, with an exchange through LDS before each (outputs written at
// their Stockham positions, the next inputs read back).  After the last pass thread t holds the
// outputs t + m n/8, stored directly: LG/3 exchanges (3 at 1024, 2 at 512) instead of a read and a
// write per pass plus the staging of the load and the store.  The passes are those of lds_fft
// (radix 2 first, then radix 8); the twiddles come from the quarter table (qtw).  C
// columns per workgroup, C n / 8 threads.
template <typename T, int DIR, bool LPRUNE, bool SPRUNE, int LG, int C>
__global__ void __launch_bounds__(C * (1 << (LG - 3))) k_fft_cols_r(ColsArgs a) {
    constexpr int N = 1 << LG, Q = N / 8, R2 = LG % 3;   // R2: a first radix-2 (1) or radix-4 (2) pass
    constexpr int PITCH = N + (N >> 3) + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V2<T>* buf = reinterpret_cast<V2<T>*>(smem_raw);
    V2<T>* tw = buf + C * PITCH;   // quarter twiddle table, w^t for t < N/4 (qtw)
    const int tid = threadIdx.x;
    const int c = tid % C, t = tid / C;
    if (a.mom && blockIdx.x == 0 && blockIdx.y == 0) finish_moments(a, blockIdx.z, C * Q);
    int cb = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0) cb = (cb & 7) * (nb >> 3) + (cb >> 3);   // XCD-contiguous column blocks
    const int o = blockIdx.y;
    const long long go = a.outer_mapped ? dmap(o, a.outer_nd, a.outer_Mr) : o;
    V2<T>* base = reinterpret_cast<V2<T>*>(a.grid) + (long long)blockIdx.z * a.gstride + go * (long long)N * a.inner +
                  band_col(a, cb) + c;   // consecutive blocks of C columns, or the blocks of a band
    V2<T> x[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int r = t + m * Q;
        x[m] = (!LPRUNE || is_data_row(r, a.nd, N)) ? base[(long long)r * a.inner] : mk<T>(0, 0);
    }
    for (int i = tid; i < N / 4; i += C * Q) tw[i] = reinterpret_cast<const V2<T>*>(a.tw)[i];
    V2<T>* line = buf + c * PITCH;
    __syncthreads();   // twiddles staged
    if constexpr (R2 == 1) {
        // pass 0, radix 2 (p = 1): butterfly i = t + Q m (m < 4) takes x[i], x[i + n/2] and writes
        // positions 2 i and 2 i + 1
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const V2<T> u = x[m], v = x[m + 4];
            const int i = t + m * Q;
            line[lpad<true>(2 * i)] = cadd<T>(u, v);
            line[lpad<true>(2 * i + 1)] = csub<T>(u, v);
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m] = line[lpad<true>(t + m * Q)];
    } else if constexpr (R2 == 2) {
        // pass 0, radix 4 (p = 1): butterfly i = t + Q m (m < 2) takes x[i + k n/4] (registers
        // m + 2 k) and writes positions 4 i + r
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            V2<T> a0 = x[m], a1 = x[m + 2], a2 = x[m + 4], a3 = x[m + 6];
            dft4<T, DIR>(a0, a1, a2, a3);
            const int i = t + m * Q;
            line[lpad<true>(4 * i)] = a0;
            line[lpad<true>(4 * i + 1)] = a1;
            line[lpad<true>(4 * i + 2)] = a2;
            line[lpad<true>(4 * i + 3)] = a3;
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m] = line[lpad<true>(t + m * Q)];
    }
    // radix-8 passes, p = 2^R2 8^s: butterfly t reads x[t + Q m] and writes (t - k) 8 + k + m p
    constexpr int NP = LG / 3;
#pragma unroll
    for (int s = 0; s < NP; ++s) {
        const int lgp = R2 + 3 * s, p = 1 << lgp, k = t & (p - 1);
        if (p > 1) {
            const int lts = LG - 3 - lgp;   // twiddle stride n / (8 p)
#pragma unroll
            for (int m = 1; m < 8; ++m) {
                V2<T> w = qtw<T, LG>(tw, (m * k) << lts);
                if (DIR > 0) w.y = -w.y;
                x[m] = cmul<T>(x[m], w);
            }
        }
        dft8<T, DIR>(x);
        if (s + 1 < NP) {
            const int j = (t - k) * 8 + k;
            __syncthreads();   // the previous reads are done
#pragma unroll
            for (int m = 0; m < 8; ++m) line[lpad<true>(j + m * p)] = x[m];
            __syncthreads();
#pragma unroll
            for (int m = 0; m < 8; ++m) x[m] = line[lpad<true>(t + m * Q)];
        }
    }
    const int nds = a.nd_store > 0 ? a.nd_store : a.nd;
#pragma unroll
    for (int m = 0; m < 8; ++m) {   // outputs t + Q m
        const int r = t + m * Q;
        if (!SPRUNE || is_data_row(r, nds, N)) base[(long long)r * a.inner] = x[m];
    }
}

// 512 threads per workgroup: 4 columns of 1024 points (64-byte row segments) or 8 of 512 (128
// bytes); 256 threads for the shorter columns: 8 of 256, 16 of 128, 32 of 64 points
template <int LG> constexpr int cols_r_c() { return LG == 10 ? 4 : LG == 9 ? 8 : 2048 >> LG; }

template <typename T, int DIR, bool LP, bool SP, int LG>
static int launch_cols_r(nlf_plan* p, ColsArgs a, int outer, int batch) {
    constexpr int C = cols_r_c<LG>(), N = 1 << LG;
    a.lg = LG;
    a.C = C;
    if (a.bc2 && (a.bc2 % C || 2 * a.bc2 > (a.bc1 ? a.Mr2 : a.inner) || (a.bc1 && 2 * a.bc1 > a.Mr1)))
        return set_error(NLF_EINVAL, "column band %d/%d does not fit the grid", a.bc1, a.bc2);
    a.ncb = a.bc2 ? (a.bc1 ? 2 * a.bc1 : 1) * (2 * a.bc2 / C) : (int)(a.inner / C);
    dim3 grid(a.ncb, outer, batch);
    const size_t lds = ((size_t)C * (N + (N >> 3) + 1) + N / 4) * sizeof(V2<T>);
    static std::mutex attr_mu;
    static bool raised = false;
    {
        std::lock_guard<std::mutex> lock(attr_mu);
        if (!raised) {
            NLF_HIP(hipFuncSetAttribute((const void*)&k_fft_cols_r<T, DIR, LP, SP, LG, C>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            raised = true;
        }
    }
    hipLaunchKernelGGL((k_fft_cols_r<T, DIR, LP, SP, LG, C>), grid, dim3(C * N / 8), lds, p->stream, a);
    NLF_HIP(hipGetLastError());
    return NLF_OK;
}

template <typename T, int DIR, bool LP, bool SP>
static int launch_cols(nlf_plan* p, ColsArgs a, int outer, int batch) {
    if (recorder() && a.n <= 512)   // recorded for the persistent executor
        return launch_cols_cfg<T, DIR, LP, SP, ExecColCfg::NT, ExecColCfg::E, true>(p, a, outer, batch);
    // lines in registers (also the band columns of a split's ball, when the band is whole blocks:
    // measured at 256^3, the ball's four band passes 60 + 27 + 28 + 59 us in LDS, 40 + 19 + 20 + 40
    // in registers; never recorded)
    if (!recorder()) {
        if (a.n == 512 && a.inner % cols_r_c<9>() == 0 && a.bc2 % cols_r_c<9>() == 0)
            return launch_cols_r<T, DIR, LP, SP, 9>(p, a, outer, batch);
        if (a.n == 1024 && a.inner % cols_r_c<10>() == 0 && a.bc2 % cols_r_c<10>() == 0)
            return launch_cols_r<T, DIR, LP, SP, 10>(p, a, outer, batch);
        // 64- to 256-point columns (also where the blocks of C columns do not fill the device: the
        // LDS kernel below takes 4096 elements per workgroup, so it would have half as many)
        auto fills = [&](int c) { return !a.bc2 && a.inner % c == 0; };
        if (a.n == 256 && fills(cols_r_c<8>())) return launch_cols_r<T, DIR, LP, SP, 8>(p, a, outer, batch);
        if (a.n == 128 && fills(cols_r_c<7>())) return launch_cols_r<T, DIR, LP, SP, 7>(p, a, outer, batch);
        if (a.n == 64 && fills(cols_r_c<6>())) return launch_cols_r<T, DIR, LP, SP, 6>(p, a, outer, batch);
    }
    if (a.n <= 512)
        return launch_cols_cfg<T, DIR, LP, SP, ColSmallCfg::NT, ColSmallCfg::E, true>(p, a, outer, batch);
    if (a.n == 1024)
        return launch_cols_cfg<T, DIR, LP, SP, Col1024Cfg::NT, Col1024Cfg::E, Col1024Cfg::TWL>(p, a, outer, batch);
    return launch_cols_cfg<T, DIR, LP, SP, FftCfg<T>::NT, FftCfg<T>::E, false>(p, a, outer, batch);
}

// The fused axis-0 pass of a split's I1 with the lines in registers, for columns of n = 8^P points
// (512 at 256^3).  Thread t of a column holds the 8 elements t + m n/8 (m = 0..7) of its line, which
// are exactly the inputs of a radix-8 Stockham butterfly of the first pass; between passes the
// outputs go through LDS once (written at their Stockham positions, read back as the next pass's
// inputs).  After the last forward pass thread t holds the frequencies t + m n/8, which are again
// the inverse transform's first inputs: the multiply by w and both transforms share registers, and
// LDS carries only the 2 (P - 1) exchanges, instead of a read and a write per pass plus the staging
// of the load, the multiply and the store.  C columns per workgroup, 64 n / 512 threads each.
// Measured at 256^3 (split potential, ms, FP64 / FP32): C = 8 2.295 / 1.205, C = 4 2.26 / 1.18.
// Tried and not kept: the passes' twiddles staged as [pass][m][k] (no LDS bank conflicts on the
// twiddle reads, 9 KiB instead of 4 KiB of LDS): 2.41 / 1.38, in every register-resident kernel;
// the real and imaginary parts exchanged in turn through half the LDS (as k_fft_rows_rw does, more
// resident workgroups but twice the barriers): this kernel 421 -> 445 us, the 512-point columns
// unchanged.
constexpr int kConv0rC = 4;   // columns per workgroup of k_fft_conv0r (64-byte row segments)

template <typename T, int P, int C>
__global__ void __launch_bounds__(C * (1 << (3 * P - 3)), 4) k_fft_conv0r(ColsArgs a, ConvW cw) {
    constexpr int LG = 3 * P, N = 1 << LG, Q = N / 8;   // line length, threads (butterflies) per line
    constexpr int PITCH = N + (N >> 3) + 1;             // padded line (one slot per 8) + 1
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V2<T>* buf = reinterpret_cast<V2<T>*>(smem_raw);
    V2<T>* tw = buf + C * PITCH;                        // quarter twiddle table, w^t for t < N/4
    const int tid = threadIdx.x;
    const int c = tid % C, t = tid / C;                 // C adjacent columns per row segment
    int cb = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0) cb = (cb & 7) * (nb >> 3) + (cb >> 3);   // XCD-contiguous column blocks
    const long long col = (long long)cb * C + c;
    V2<T>* base = reinterpret_cast<V2<T>*>(a.grid) + (long long)blockIdx.z * a.gstride + col;
    V2<T> x[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {   // the data rows of the padded column; the rest are zero
        const int r = t + m * Q;
        x[m] = is_data_row(r, a.nd, N) ? base[(long long)r * a.inner] : mk<T>(0, 0);
    }
    for (int i = tid; i < N / 4; i += C * Q) tw[i] = reinterpret_cast<const V2<T>*>(a.tw)[i];
    V2<T>* line = buf + c * PITCH;
    // one radix-8 pass on the registers: butterfly t, p = 8^s, inputs x[m] = line[t + m Q]
    auto pass = [&](int s, auto dir) {
        constexpr int DIR = decltype(dir)::value;
        const int p = 1 << (3 * s), k = t & (p - 1);
        if (s > 0) {
            const int lts = LG - 3 - 3 * s;   // twiddle stride n / (8 p)
#pragma unroll
            for (int m = 1; m < 8; ++m) {
                V2<T> w = qtw<T, LG>(tw, (m * k) << lts);
                if (DIR > 0) w.y = -w.y;
                x[m] = cmul<T>(x[m], w);
            }
        }
        dft8<T, DIR>(x);
    };
    // outputs of pass s to their Stockham positions, then the next pass's inputs
    auto exchange = [&](int s) {
        const int p = 1 << (3 * s), k = t & (p - 1);
        const int j = (t - k) * 8 + k;
        __syncthreads();   // the previous exchange's reads are done
#pragma unroll
        for (int m = 0; m < 8; ++m) line[lpad<true>(j + m * p)] = x[m];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m] = line[lpad<true>(t + m * Q)];
    };
    __syncthreads();   // twiddles staged
    using Fwd = std::integral_constant<int, -1>;
    using Inv = std::integral_constant<int, 1>;
    double e0[8];   // the multiply's row factors (a small table, read through the caches)
#pragma unroll
    for (int s = 0; s < P; ++s) {
        if (s + 1 == P) {
#pragma unroll
            for (int m = 0; m < 8; ++m) e0[m] = cw.e0[t + m * Q];
        }
        pass(s, Fwd{});
        if (s + 1 < P) exchange(s);
    }
    // thread t holds frequencies t + m Q: multiply by w(k) (column terms once per thread, the
    // row factor exp(-k0^2/a) from the plan's table; expm1 where 1 - e^{-x} would cancel)
    {
        const int c1 = (int)(col / cw.pitch2), c2 = (int)(col - (long long)c1 * cw.pitch2);
        const double k1 = (c1 < cw.Mr1 / 2 ? c1 : c1 - cw.Mr1) * cw.dk1;
        const double k2 = (c2 < cw.Mr2 / 2 ? c2 : c2 - cw.Mr2) * cw.dk2;
        const double q12 = k1 * k1 + k2 * k2;
        const double e12 = exp(-q12 * cw.inva);
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int r = t + m * Q;
            const double k0 = (r < cw.Mr0 / 2 ? r : r - cw.Mr0) * cw.dk0;
            const double kk = k0 * k0 + q12;
            const double xx = kk * cw.inva;
            double w;
            if (xx >= 1.0) w = (1.0 - e0[m] * e12) * rcp_newton(kk);
            else w = kk > 0.0 ? -expm1(-xx) / kk : cw.inva;
            x[m].x = (T)((double)x[m].x * w);
            x[m].y = (T)((double)x[m].y * w);
        }
    }
#pragma unroll
    for (int s = 0; s < P; ++s) {
        pass(s, Inv{});
        if (s + 1 < P) exchange(s);
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) {   // outputs t + m Q: the data rows only
        const int r = t + m * Q;
        if (is_data_row(r, a.nd, N)) base[(long long)r * a.inner] = x[m];
    }
}

template <typename T, int P, int C>
static int launch_conv0r(nlf_plan* p, ColsArgs a, ConvW cw, int batch) {
    constexpr int N = 1 << (3 * P), NT = C * N / 8;
    a.ncb = (int)(a.inner / C);
    dim3 grid(a.ncb, 1, batch);
    const size_t lds = ((size_t)C * (N + (N >> 3) + 1) + N / 4) * sizeof(V2<T>);
    static std::mutex attr_mu;
    static bool raised = false;
    {
        std::lock_guard<std::mutex> lock(attr_mu);
        if (!raised) {
            NLF_HIP(hipFuncSetAttribute((const void*)&k_fft_conv0r<T, P, C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)lds));
            raised = true;
        }
    }
    hipLaunchKernelGGL((k_fft_conv0r<T, P, C>), grid, dim3(NT), lds, p->stream, a, cw);
    NLF_HIP(hipGetLastError());
    return NLF_OK;
}

template <typename T, int NT, int E, bool TWL>
static int launch_conv0_cfg(nlf_plan* p, ColsArgs a, ConvW cw, int batch) {
    a.lg = ilog2(a.n);
    int C = 16;   // as in launch_cols_cfg
    while (C > 1 && (C * a.n > E || a.inner % C || (a.inner / C) * batch < 256)) C >>= 1;
    if (a.n + 1 > E) return set_error(NLF_EUNSUPPORTED, "FFT length %d exceeds the LDS line budget", a.n);
    a.C = C;
    a.ncb = (int)(a.inner / C);
    dim3 grid(a.ncb, 1, batch);
    size_t lds = ((size_t)C * (lds_line(a.n, TWL) + 1) + (TWL ? a.n / 2 : 0)) * sizeof(V2<T>);   // columns (+ twiddles)
    // raised on first need; the check and the raise are one step, for plans driven from several threads
    static std::mutex attr_mu;
    static size_t attr_bytes = 0;
    {
        std::lock_guard<std::mutex> lock(attr_mu);
        if (lds > attr_bytes) {
            NLF_HIP(hipFuncSetAttribute((const void*)&k_fft_conv0<T, NT, E, TWL>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)lds));
            attr_bytes = lds;
        }
    }
    hipLaunchKernelGGL((k_fft_conv0<T, NT, E, TWL>), grid, dim3(NT), lds, p->stream, a, cw);
    NLF_HIP(hipGetLastError());
    return NLF_OK;
}

// I1 of a split (Eq. '3.9'), 3D: the cyclic convolution of the zero-padded density with the lattice
// transform of w, u += (1/G) IFFT(w . FFT(pad rho)), truncated to the data grid.  The plan's pre-
// and post-correction tables are ones, so the row and axis-1 passes are the plain padded FFT; the
// axis-0 passes and the multiply are one fused kernel.  rho is real and w real and even, so the
// spectrum is Hermitian and, after the inverse axis-0 and axis-1 passes, every line along axis 2 is
// Hermitian in its own frequency: only the first H = Mr2/2 + 16 frequencies of axis 2 are kept
// (H a multiple of the column blocks), about half the data of the axis-1 and axis-0 passes.
template <typename T>
static int split_i1_t(nlf_plan* p, const void* rho, void* u) {
    const int H = std::min(p->Mr[2], p->Mr[2] / 2 + 16);
    RowsArgs r{};
    r.grid = p->grid_a;
    r.gstride = p->G;
    r.rho = rho;
    r.rstride = p->N;
    r.n = p->Mr[2];
    r.dim = 3;
    for (int i = 0; i < 3; ++i) { r.nd[i] = p->n[i]; r.Mr[i] = p->Mr[i]; }
    r.dec0 = p->dec[0];
    r.dec1 = p->dec[1];
    r.dec2 = p->dec[2];
    r.tw = p->tw_big[2];
    r.nlines = p->n[0] * p->n[1];
    r.half = H;
    r.nonfinite = p->nf_flag;
    NLF_TRY((launch_rows<T, -1, LOAD_RHO, STORE_GRID>(p, r, p->batch)));
    ColsArgs c{};
    c.grid = p->grid_a; c.gstride = p->G; c.n = p->Mr[1]; c.inner = H;
    c.outer_mapped = 1; c.outer_nd = p->n[0]; c.outer_Mr = p->Mr[0];
    c.nd = p->n[1]; c.tw = p->tw_big[1];
    NLF_TRY((launch_cols<T, -1, true, false>(p, c, p->n[0], p->batch)));
    ColsArgs c0{};
    c0.grid = p->grid_a; c0.gstride = p->G; c0.n = p->Mr[0]; c0.inner = (long long)p->Mr[1] * H;
    c0.nd = p->n[0]; c0.tw = p->tw_big[0];
    ConvW cw{p->Mr[0], p->Mr[1], p->Mr[2], H, 0, 0, 0, 1.0 / p->split_a, p->conv_e0};
    cw.dk0 = 2.0 * 3.14159265358979323846 / (p->Mr[0] * p->h[0]);
    cw.dk1 = 2.0 * 3.14159265358979323846 / (p->Mr[1] * p->h[1]);
    cw.dk2 = 2.0 * 3.14159265358979323846 / (p->Mr[2] * p->h[2]);
    if (c0.n == 512 && c0.inner % kConv0rC == 0)   // lines in registers
        NLF_TRY((launch_conv0r<T, 3, kConv0rC>(p, c0, cw, p->batch)));
    else if (c0.n <= 512) NLF_TRY((launch_conv0_cfg<T, ColSmallCfg::NT, ColSmallCfg::E, true>(p, c0, cw, p->batch)));
    else NLF_TRY((launch_conv0_cfg<T, FftCfg<T>::NT, FftCfg<T>::E, false>(p, c0, cw, p->batch)));
    c.nd = p->n[1];
    NLF_TRY((launch_cols<T, 1, false, true>(p, c, p->n[0], p->batch)));
    RowsArgs ri = r;
    ri.rho = nullptr;
    ri.u = u;
    ri.post = p->post;
    ri.accum = 1;
    return launch_rows<T, 1, LOAD_GRID, STORE_U, T>(p, ri, p->batch);
}

int fft_split_i1(nlf_plan* p, const void* rho, void* u) {
    return p->prec == NLF_F64 ? split_i1_t<double>(p, rho, u) : split_i1_t<float>(p, rho, u);
}

template <typename T>
static int type2_forward_t(nlf_plan* p, const void* rho) {
    const int d = p->dim;
    RowsArgs r{};
    r.grid = p->grid_a;
    r.gstride = p->G;
    r.rho = rho;
    r.rstride = p->N;
    r.n = p->Mr[d - 1];
    r.dim = d;
    for (int i = 0; i < 3; ++i) { r.nd[i] = p->n[i]; r.Mr[i] = p->Mr[i]; }
    r.dec0 = p->dec[0];
    r.dec1 = p->dec[1];
    r.dec2 = p->dec[2];
    r.tw = p->tw_big[d - 1];
    r.nlines = (d == 2) ? p->n[0] : p->n[0] * p->n[1];
    r.band = p->band;
    r.nonfinite = p->nf_flag;
    // 2D Laplace: the moments m0, m1 of rho (Alg. 1) ride along the row pass
    const bool mom = (p->kernel == NLF_LAPLACE2D);
    if (mom) {
        r.mom_part = p->red;
        r.L0 = p->L[0]; r.L1 = p->L[1]; r.h0 = p->h[0]; r.h1 = p->h[1];
    }
    NLF_TRY((launch_rows<T, -1, LOAD_RHO, STORE_GRID>(p, r, p->batch)));
    if (d == 2) {
        ColsArgs c{};
        c.grid = p->grid_a; c.gstride = p->G; c.n = p->Mr[0]; c.inner = p->Mr[1];
        c.nd = p->n[0]; c.tw = p->tw_big[0];
        if (mom) {
            const int lpw = rows_lines_per_wg(p->Mr[1]);   // the row pass's grid
            c.mom_part = p->red;
            c.mom_nblk = (p->n[0] + lpw - 1) / lpw;
            c.mom_w = p->h[0] * p->h[1];
            c.mom = p->mom;
        }
        NLF_TRY((launch_cols<T, -1, true, false>(p, c, 1, p->batch)));
    } else if (p->band) {
        // the ball of a split: only the band |f_i| < band of the spectrum is interpolated
        ColsArgs c{};
        c.grid = p->grid_a; c.gstride = p->G; c.n = p->Mr[1]; c.inner = p->Mr[2];
        c.outer_mapped = 1; c.outer_nd = p->n[0]; c.outer_Mr = p->Mr[0];
        c.nd = p->n[1]; c.nd_store = 2 * p->band; c.tw = p->tw_big[1];
        c.bc2 = p->band; c.Mr2 = p->Mr[2];
        NLF_TRY((launch_cols<T, -1, true, true>(p, c, p->n[0], p->batch)));
        ColsArgs c0{};
        c0.grid = p->grid_a; c0.gstride = p->G; c0.n = p->Mr[0]; c0.inner = (long long)p->Mr[1] * p->Mr[2];
        c0.nd = p->n[0]; c0.nd_store = 2 * p->band; c0.tw = p->tw_big[0];
        c0.bc1 = p->band; c0.bc2 = p->band; c0.Mr1 = p->Mr[1]; c0.Mr2 = p->Mr[2];
        NLF_TRY((launch_cols<T, -1, true, true>(p, c0, 1, p->batch)));
    } else {
        ColsArgs c{};
        c.grid = p->grid_a; c.gstride = p->G; c.n = p->Mr[1]; c.inner = p->Mr[2];
        c.outer_mapped = 1; c.outer_nd = p->n[0]; c.outer_Mr = p->Mr[0];
        c.nd = p->n[1]; c.tw = p->tw_big[1];
        NLF_TRY((launch_cols<T, -1, true, false>(p, c, p->n[0], p->batch)));
        ColsArgs c0{};
        c0.grid = p->grid_a; c0.gstride = p->G; c0.n = p->Mr[0]; c0.inner = (long long)p->Mr[1] * p->Mr[2];
        c0.nd = p->n[0]; c0.tw = p->tw_big[0];
        NLF_TRY((launch_cols<T, -1, true, false>(p, c0, 1, p->batch)));
    }
    return NLF_OK;
}

template <typename T, typename TU>
static int type1_inverse_t(nlf_plan* p, void* u, bool add_u1) {
    const int d = p->dim;
    if (d == 2) {
        ColsArgs c{};
        c.grid = p->grid_b; c.gstride = p->G; c.n = p->Mr[0]; c.inner = p->Mr[1];
        c.nd = p->n[0]; c.tw = p->tw_t1[0];
        NLF_TRY((launch_cols<T, 1, false, true>(p, c, 1, p->batch)));
    } else if (p->band) {
        // the ball of a split: the spreading grid is zero outside the band |f_i| < band
        ColsArgs c0{};
        c0.grid = p->grid_b; c0.gstride = p->G; c0.n = p->Mr[0]; c0.inner = (long long)p->Mr[1] * p->Mr[2];
        c0.nd = 2 * p->band; c0.nd_store = p->n[0]; c0.tw = p->tw_t1[0];
        c0.bc1 = p->band; c0.bc2 = p->band; c0.Mr1 = p->Mr[1]; c0.Mr2 = p->Mr[2];
        NLF_TRY((launch_cols<T, 1, true, true>(p, c0, 1, p->batch)));
        ColsArgs c{};
        c.grid = p->grid_b; c.gstride = p->G; c.n = p->Mr[1]; c.inner = p->Mr[2];
        c.outer_mapped = 1; c.outer_nd = p->n[0]; c.outer_Mr = p->Mr[0];
        c.nd = 2 * p->band; c.nd_store = p->n[1]; c.tw = p->tw_t1[1];
        c.bc2 = p->band; c.Mr2 = p->Mr[2];
        NLF_TRY((launch_cols<T, 1, true, true>(p, c, p->n[0], p->batch)));
    } else {
        ColsArgs c0{};
        c0.grid = p->grid_b; c0.gstride = p->G; c0.n = p->Mr[0]; c0.inner = (long long)p->Mr[1] * p->Mr[2];
        c0.nd = p->n[0]; c0.tw = p->tw_t1[0];
        NLF_TRY((launch_cols<T, 1, false, true>(p, c0, 1, p->batch)));
        ColsArgs c{};
        c.grid = p->grid_b; c.gstride = p->G; c.n = p->Mr[1]; c.inner = p->Mr[2];
        c.outer_mapped = 1; c.outer_nd = p->n[0]; c.outer_Mr = p->Mr[0];
        c.nd = p->n[1]; c.tw = p->tw_t1[1];
        NLF_TRY((launch_cols<T, 1, false, true>(p, c, p->n[0], p->batch)));
    }
    RowsArgs r{};
    r.grid = p->grid_b;
    r.gstride = p->G;
    r.u = u;
    r.rstride = p->N;
    r.n = p->Mr[d - 1];
    r.dim = d;
    for (int i = 0; i < 3; ++i) { r.nd[i] = p->n[i]; r.Mr[i] = p->Mr[i]; }
    r.dec0 = p->dec[0];
    r.dec1 = p->dec[1];
    r.dec2 = p->dec[2];
    r.tw = p->tw_t1[d - 1];
    r.post = p->post;
    r.band = p->band;
    r.nlines = (d == 2) ? p->n[0] : p->n[0] * p->n[1];
    r.add_u1 = add_u1 ? 1 : 0;
    r.mom = p->mom;
    r.u11 = p->u11;
    r.sigma = p->sigma;
    r.L0 = p->L[0];
    r.L1 = p->L[1];
    r.h0 = p->h[0];
    r.h1 = p->h[1];
    return launch_rows<T, 1, LOAD_GRID, STORE_U, TU>(p, r, p->batch);
}

int fft_type2_forward(nlf_plan* p, const void* rho) {
    return p->prec == NLF_F64 ? type2_forward_t<double>(p, rho) : type2_forward_t<float>(p, rho);
}

int fft_type1_inverse(nlf_plan* p, void* u, bool add_u1) {
    if (p->prec == NLF_F64) return type1_inverse_t<double, double>(p, u, add_u1);
    if (p->t1_prec == NLF_F64) return type1_inverse_t<double, float>(p, u, add_u1);
    return type1_inverse_t<float, float>(p, u, add_u1);
}

// Full complex FFT of [batch][n] fields on the plan's (non-oversampled) grid, in place.
template <typename T, int DIR>
static int full_t(nlf_plan* p, void* data, int batch) {
    const int d = p->dim;
    RowsArgs r{};
    r.grid = data;
    r.gstride = p->N;
    r.n = p->n[d - 1];
    r.dim = d;
    r.tw = p->tw_small[d - 1];
    r.nlines = (int)(p->N / p->n[d - 1]);
    NLF_TRY((launch_rows<T, DIR, LOAD_GRID, STORE_GRID>(p, r, batch)));
    if (d == 3) {
        ColsArgs c{};
        c.grid = data; c.gstride = p->N; c.n = p->n[1]; c.inner = p->n[2]; c.nd = p->n[1];
        c.tw = p->tw_small[1];
        NLF_TRY((launch_cols<T, DIR, false, false>(p, c, p->n[0], batch)));
    }
    ColsArgs c0{};
    c0.grid = data; c0.gstride = p->N; c0.n = p->n[0];
    c0.inner = (d == 2) ? p->n[1] : (long long)p->n[1] * p->n[2];
    c0.nd = p->n[0];
    c0.tw = p->tw_small[0];
    return launch_cols<T, DIR, false, false>(p, c0, 1, batch);
}

int fft_full(nlf_plan* p, void* data, int dir, int batch) {
    if (p->prec == NLF_F64) return dir < 0 ? full_t<double, -1>(p, data, batch) : full_t<double, 1>(p, data, batch);
    return dir < 0 ? full_t<float, -1>(p, data, batch) : full_t<float, 1>(p, data, batch);
}

__global__ void k_clear_flag(int* f) { *f = 0; }

// Wait for the plan's work, read the density load pass's non-finite flag into *seen and clear it.
int read_nonfinite(nlf_plan* p, int* seen) {
    int v = 0;
    NLF_HIP(hipMemcpyAsync(&v, p->nf_flag, sizeof(int), hipMemcpyDeviceToHost, p->stream));
    NLF_HIP(hipStreamSynchronize(p->stream));
    *seen = v;
    if (v) {
        hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, p->stream, p->nf_flag);
        NLF_HIP(hipGetLastError());
    }
    return NLF_OK;
}

int fill_zero(nlf_plan* p, void* ptr, size_t bytes) {
    // device buffers of the plan are 256-byte aligned; sizes are multiples of 8 bytes
    const long long n16 = (long long)(bytes / 16);
    if (n16 > 0) {
        const int blocks = (int)std::max<long long>(1, std::min<long long>((n16 + 1023) / 1024, 2048));
        hipLaunchKernelGGL(k_fill_zero16, dim3(blocks), dim3(256), 0, p->stream, (double2*)ptr, n16);
    }
    if (bytes % 16)
        hipLaunchKernelGGL((k_fill_zero<double>), dim3(1), dim3(64), 0, p->stream, (double*)ptr + 2 * n16,
                           (long long)((bytes % 16) / 8));
    NLF_HIP(hipGetLastError());
    return NLF_OK;
}

}  // namespace nlf
